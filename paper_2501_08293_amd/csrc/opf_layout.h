// Host-side data layout of the componentwise ADMM (internal header).
//
// Components are packed into 64-lane wavefronts: every lane of a wavefront
// owns one local slot (one row of its component's projection), a component
// never straddles two wavefronts, and the factor rows of a wavefront are
// stored k-major ([k][lane]) so that the k-th column read by all 64 lanes is
// one contiguous 512-byte (FP64) segment.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace opf {

constexpr int kWave = 64;

struct ProblemView {
    int32_t n = 0, S = 0;
    const double* c = nullptr;
    const double* lb = nullptr;
    const double* ub = nullptr;
    const uint8_t* var_kind = nullptr;
    const int32_t* comp_m = nullptr;
    const int32_t* comp_n = nullptr;
    const double* A = nullptr;
    const double* b = nullptr;
    const int32_t* idx = nullptr;
};

struct HostLayout {
    int32_t n = 0, S = 0, L = 0;
    int32_t waves = 0;          // packed wavefronts (blocks * block_waves, some may be empty)
    int32_t block_waves = 0;    // wavefronts per workgroup (input: requested, 0 = default)
    int32_t blocks = 0;         // workgroups
    int32_t max_nbrs = 0;       // largest neighbour list
    int32_t max_ns = 0, max_copies = 0;
    int64_t sum_ns2 = 0;
    bool factors_on_device = false;   // input: leave F and bbar empty (computed by the device set-up)
    std::vector<int8_t> comp_group;   // input (optional, per component): components of group 1 come
                                      // first and never share a wavefront with group 0

    // per wavefront
    std::vector<int32_t> wave_maxn;   // columns stored for the wavefront
    std::vector<int64_t> wave_foff;   // element offset of its factor block

    // per lane (device slot d = wave * 64 + lane); padding lanes have var = -1
    std::vector<int32_t> var;         // global variable copied by the slot
    std::vector<int32_t> meta;        // base lane | n_s << 8 | (owner flag) << 16
    std::vector<int32_t> copy_start;  // offset into copy_list
    std::vector<int32_t> copy_cnt;    // number of copies of var (N_i)
    std::vector<int32_t> user_slot;   // user slot order index, -1 for padding
    std::vector<double>  bbar;        // bbar_s entry of the slot
    std::vector<double>  lo, hi, cost;   // bounds and objective of var, per slot
    std::vector<double>  z0;          // default initial local copy (Section V-A)

    std::vector<int32_t> user_to_dev; // [L]
    std::vector<int32_t> owner_slot;  // [n] device slot that writes x_i
    std::vector<int32_t> copy_list;   // per slot: all copies of its variable, ascending

    std::vector<double> F;            // packed factors F_s = I - P_s, [k][lane] per wave

    // workgroups owning a copy of a variable of workgroup b: nbr_list[nbr_ptr[b] .. nbr_ptr[b+1])
    std::vector<int32_t> nbr_ptr;
    std::vector<int32_t> nbr_list;

    std::vector<double> c_full;       // [n] objective (for c^T x)

    // per component (filled when factors_on_device): first device slot
    // (wave * 64 + base lane), offsets of its A block and b entries
    std::vector<int32_t> comp_dev;
    std::vector<int64_t> comp_aoff, comp_boff;
};

// Returns 0 or an OPF_E* code with a message in err.
int build_layout(const ProblemView& p, HostLayout& out, std::string& err, int threads);

// Factor of one component: F = I - A^T (A A^T)^{-1} A and bbar = A^T (A A^T)^{-1} b
// from the row-reduced [A | b].  Row-major n x n F.  Returns 0, or
// OPF_EINFEASIBLE_COMPONENT when row reduction finds 0 = nonzero.
int component_factor(int m, int n, const double* A, const double* b, double* F, double* bbar,
                     int* rank_out);

// The same for r right-hand sides at once: Bm is m x r row-major, bbar n x r.
// With r_in < 0 the |r_in| right-hand sides are not checked for consistency.
int component_factor_multi(int m, int n, const double* A, int r_in, const double* Bm, double* F,
                           double* bbar, int* rank_out);

// Linear map b -> bbar of one component (n x m row-major): bbar = Wmap b for
// every right-hand side consistent with A.
int component_rhs_map(int m, int n, const double* A, double* F, double* Wmap);

// Batched scenarios sharing A: bbar of every slot and scenario in device order,
// [slot][Kp] (scenario-minor, Kp >= K padded with zeros).  b_scen is [K][sum m_s].
int build_batch_rhs(const ProblemView& p, const HostLayout& lay, const double* b_scen, int K, int Kp,
                    std::vector<float>& out, std::string& err, int threads,
                    const std::vector<int8_t>* skip = nullptr);

// Dense block-diagonal 64 x 64 factor of every wavefront (row = output lane,
// column = input lane), split into `terms` bfloat16 planes whose sum
// approximates F: plane t holds bf16(F - sum of planes < t).  Layout
// [terms][wave][64][64].
void build_dense_planes(const HostLayout& lay, int terms, std::vector<uint16_t>& planes);

}  // namespace opf
