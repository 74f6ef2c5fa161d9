// Host-only driver for the library's set-up code (validation, row reduction,
// factors, packing): reads a problem from a raw binary file, builds the layout
// and writes it back for invariant checks.  Built with g++ (optionally with
// AddressSanitizer/UBSan); no GPU involved.
//
// input:  int32 n, S, B; then c[n], lb[n], ub[n] (f64); var_kind[n] (u8);
//         comp_m[S], comp_n[S] (i32); A (f64, sum m*n); b (f64, sum m); idx (i32, sum n)
// output: int32 rc, n, S, L, waves, blocks, B, max_nbrs; then var, meta, user_slot,
//         copy_start, copy_cnt (i32, waves*64 each); copy_list (i32, L); wave_maxn (i32, waves);
//         wave_foff (i64, waves); F (f64); bbar (f64, waves*64); nbr_ptr (i32, blocks+1); nbr_list
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_2501_08293_amd/csrc/opf_layout.h"

template <typename T>
static void rd(FILE* f, std::vector<T>& v, size_t n) {
    v.resize(n);
    if (n && fread(v.data(), sizeof(T), n, f) != n) { fprintf(stderr, "short read\n"); exit(2); }
}
template <typename T>
static void wr(FILE* f, const std::vector<T>& v) {
    if (!v.empty()) fwrite(v.data(), sizeof(T), v.size(), f);
}

int main(int argc, char** argv) {
    if (argc < 3) { fprintf(stderr, "usage: layout_driver in.bin out.bin\n"); return 2; }
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t hdr[3];
    if (fread(hdr, 4, 3, f) != 3) return 2;
    const int n = hdr[0], S = hdr[1], B = hdr[2];
    std::vector<double> c, lb, ub, A, b;
    std::vector<uint8_t> kind;
    std::vector<int32_t> cm, cn, idx;
    rd(f, c, n); rd(f, lb, n); rd(f, ub, n); rd(f, kind, n); rd(f, cm, S); rd(f, cn, S);
    size_t na = 0, nb = 0, ni = 0;
    for (int s = 0; s < S; ++s) { na += (size_t)cm[s] * cn[s]; nb += cm[s]; ni += cn[s]; }
    rd(f, A, na); rd(f, b, nb); rd(f, idx, ni);
    fclose(f);
    opf::ProblemView v;
    v.n = n; v.S = S; v.c = c.data(); v.lb = lb.data(); v.ub = ub.data(); v.var_kind = kind.data();
    v.comp_m = cm.data(); v.comp_n = cn.data(); v.A = A.data(); v.b = b.data(); v.idx = idx.data();
    opf::HostLayout L;
    L.block_waves = B;
    std::string err;
    const int rc = opf::build_layout(v, L, err, 4);
    FILE* o = fopen(argv[2], "wb");
    int32_t out[8] = {rc, L.n, L.S, L.L, L.waves, L.blocks, L.block_waves, L.max_nbrs};
    fwrite(out, 4, 8, o);
    if (rc == 0) {
        wr(o, L.var); wr(o, L.meta); wr(o, L.user_slot); wr(o, L.copy_start); wr(o, L.copy_cnt);
        wr(o, L.copy_list); wr(o, L.wave_maxn); wr(o, L.wave_foff); wr(o, L.F); wr(o, L.bbar);
        wr(o, L.nbr_ptr); wr(o, L.nbr_list);
    } else {
        fprintf(stderr, "%s\n", err.c_str());
    }
    fclose(o);
    return 0;
}
