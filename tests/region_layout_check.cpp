// Host-only check of the compact region layout's half layout of B (no GPU):
// reads a system and a region list, builds the layout with the library's own
// builder and verifies, region by region, against the full layout built
// beside it:
//   - every off-diagonal pair {p, q} of B's full rows is stored exactly once,
//     in the row the split rule names, with the same FP32 value;
//   - the diagonal per position (zero on padding positions);
//   - padding entries (weight zero on the row's own position) only past a
//     row's stored pairs, and each slice's length = its longest half row;
//   - the fixed-point bound: max |value| x (most transpose terms of a
//     position) < 2^heb, so no 32-bit sum of terms below 2^(30 - L) overflows.
// Input (binary, little endian): int32 N, int64 nnzb, int64 nnz, double box,
// int8 n_orb[N], int64 blk_row_ptr[N+1], int32 blk_col[nnzb],
// int64 val_ptr[nnzb+1], double A[nnz], double B[nnz], double pos[3N],
// int32 n_regions, int32 centres[n_regions], double radii[n_regions].
// Prints one line of statistics (with the most transpose terms any position
// takes), then per region "ritz r lo hi" (the extreme
// Ritz values of its B from the builder's Lanczos), and exits 0, or names the
// first failure.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <map>
#include <vector>

#include "internal.h"

namespace {

template <typename T>
bool rd(FILE* f, T* p, size_t n) {
    return fread(p, sizeof(T), n, f) == n;
}

int fail(const char* what, int r, int p, int q) {
    printf("FAIL region %d position %d / %d: %s\n", r, p, q, what);
    return 1;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s input.bin\n", argv[0]);
        return 2;
    }
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t N = 0;
    int64_t nnzb = 0, nnz = 0;
    double box = 0;
    bool ok = rd(f, &N, 1) && rd(f, &nnzb, 1) && rd(f, &nnz, 1) && rd(f, &box, 1);
    std::vector<int8_t> n_orb(N);
    std::vector<int64_t> rp(N + 1), vp(nnzb + 1);
    std::vector<int32_t> bc(nnzb);
    std::vector<double> A(nnz), B(nnz), pos(3 * (size_t)N);
    ok = ok && rd(f, n_orb.data(), N) && rd(f, rp.data(), N + 1) && rd(f, bc.data(), nnzb) &&
         rd(f, vp.data(), nnzb + 1) && rd(f, A.data(), nnz) && rd(f, B.data(), nnz) && rd(f, pos.data(), 3 * N);
    int32_t nr = 0;
    ok = ok && rd(f, &nr, 1);
    std::vector<int32_t> centres(nr);
    std::vector<double> radii(nr);
    ok = ok && rd(f, centres.data(), nr) && rd(f, radii.data(), nr);
    fclose(f);
    if (!ok) return 2;

    elses::HostMatrix h;
    h.n_atoms = N;
    h.atom_off.assign(N + 1, 0);
    for (int I = 0; I < N; ++I) h.atom_off[I + 1] = h.atom_off[I] + n_orb[I];
    h.M = h.atom_off[N];
    h.brow.assign(rp.begin(), rp.end());
    h.bcol.assign(bc.begin(), bc.end());
    h.atom_plen.assign(N, 0);
    for (int I = 0; I < N; ++I) {
        for (int64_t b = rp[I]; b < rp[I + 1]; ++b) h.atom_plen[I] += n_orb[bc[b]];
        h.pmax = std::max(h.pmax, h.atom_plen[I]);
    }
    h.pos = pos;
    h.box = box;
    h.n_orb = n_orb;
    h.in_voff = vp;
    h.A_in = A;
    h.B_in = B;

    elses::CompactHost C;
    const char* err = elses::build_compact(h, nr, centres.data(), radii.data(), nullptr, true, C);
    if (err) {
        printf("FAIL build: %s\n", err);
        return 1;
    }
    int64_t pairs_total = 0, slots_total = 0;
    double worst_fill = 1.0;
    int fan_most = 0;
    for (int r = 0; r < nr; ++r) {
        const elses::RegionDesc& D = C.reg[r];
        const int P = D.nslice * 64;
        // full layout: off-diagonal pairs (lower position first) and the diagonal
        std::map<std::pair<int, int>, float> full;
        std::vector<float> diag(P, 0.0f);
        for (int s = 0; s < D.nslice; ++s) {
            const int len = C.slice_len[D.slice0 + s];
            const int64_t e0 = D.ent0 + C.slice_ent[D.slice0 + s];
            for (int l = 0; l < 64; ++l) {
                const int p = 64 * s + l;
                for (int k = 0; k < len; ++k) {
                    const int64_t e = e0 + (int64_t)k * 64 + l;
                    const int q = C.idx[e];
                    const float b = C.B32[e];
                    if (q == p) {
                        if (b != 0.0f) diag[p] = b;  // padding carries weight zero
                        continue;
                    }
                    const auto key = std::make_pair(std::min(p, q), std::max(p, q));
                    const auto it = full.find(key);
                    if (it == full.end())
                        full[key] = b;
                    else if (it->second != b)
                        return fail("full layout not symmetric", r, p, q);
                }
            }
        }
        // half layout
        std::map<std::pair<int, int>, float> half;
        std::vector<int> fan(P, 0);
        float bmax = 0.0f;
        int64_t slots = 0;
        for (int s = 0; s < D.nslice; ++s) {
            const int len = C.hslice_len[D.slice0 + s];
            const int64_t e0 = D.hent0 + C.hslice_ent[D.slice0 + s];
            int longest = 0;
            for (int l = 0; l < 64; ++l) {
                const int p = 64 * s + l;
                bool padding = false;
                int n = 0;
                for (int k = 0; k < len; ++k) {
                    const int64_t e = e0 + (int64_t)k * 64 + l;
                    const int q = C.hidx[e];
                    const float b = C.hval[e];
                    if (q == p && b == 0.0f) {
                        padding = true;
                        continue;
                    }
                    if (padding) return fail("stored pair after padding", r, p, q);
                    if (q == p) return fail("diagonal in the half rows", r, p, q);
                    const bool owner = ((p + q) & 1) == 0 ? (p < q) : (p > q);
                    if (!owner) return fail("pair stored in the wrong row", r, p, q);
                    const auto key = std::make_pair(std::min(p, q), std::max(p, q));
                    if (half.count(key)) return fail("pair stored twice", r, p, q);
                    half[key] = b;
                    ++fan[q];
                    bmax = std::max(bmax, std::fabs(b));
                    ++n;
                }
                longest = std::max(longest, n);
            }
            if (longest != len) return fail("slice length is not its longest half row", r, 64 * s, len);
            slots += (int64_t)len * 64;
        }
        if (half.size() != full.size()) return fail("half layout misses pairs", r, (int)half.size(), (int)full.size());
        for (const auto& kv : full) {
            const auto it = half.find(kv.first);
            if (it == half.end()) return fail("pair missing from the half layout", r, kv.first.first, kv.first.second);
            if (it->second != kv.second) return fail("value differs", r, kv.first.first, kv.first.second);
        }
        for (int p = 0; p < P; ++p)
            if (C.hdiag[D.pos0 + p] != diag[p]) return fail("diagonal differs", r, p, p);
        if (C.region_hnnz[r] != (int64_t)half.size()) return fail("stored-pair count", r, 0, 0);
        int fmax = 0;
        for (int x : fan) fmax = std::max(fmax, x);
        if (!((double)bmax * (fmax + 1) < std::ldexp(1.0, D.heb)))
            return fail("fixed-point bound", r, fmax, D.heb);
        fan_most = std::max(fan_most, fmax);
        pairs_total += (int64_t)half.size();
        slots_total += slots;
        if (slots > 0) worst_fill = std::min(worst_fill, (double)half.size() / (double)slots);
    }
    printf("ok regions %d pairs %lld slots %lld fill %.4f worst %.4f fan %d\n", nr, (long long)pairs_total,
           (long long)slots_total, slots_total ? (double)pairs_total / (double)slots_total : 1.0, worst_fill,
           fan_most);
    for (int r = 0; r < nr; ++r) printf("ritz %d %.17g %.17g\n", r, C.ritz_lo[r], C.ritz_hi[r]);
    return 0;
}
