// Host-side construction of the compact per-region layout (see region.hip).
//
// Region r is the set of atoms whose minimum-image distance to the centre
// atom is <= radius (the paper's real-space projection, Sec. III-B, with a
// radius in place of an atom count), in ascending atom order; its matrices
// are the principal sub-blocks of A and B on those atoms.  The build runs on
// all host threads: a cell list finds each region's atoms, then every region
// is laid out independently into pre-computed offsets.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <functional>
#include <thread>

#include "internal.h"

namespace elses {

namespace {

// Cell list of a periodic cube (or none: every query scans all atoms).
struct Cells {
    int nc = 0;
    double side = 0;
    std::vector<int> start, atoms;
};

Cells make_cells(const HostMatrix& h) {
    Cells c;
    if (!(h.box > 0.0)) return c;
    int nc = (int)std::floor(h.box / 4.0);
    nc = std::max(1, std::min(nc, 128));
    c.nc = nc;
    c.side = h.box / nc;
    const int N = h.n_atoms;
    std::vector<int> key(N);
    for (int I = 0; I < N; ++I) {
        int k[3];
        for (int d = 0; d < 3; ++d) {
            double p = std::fmod(h.pos[3 * I + d], h.box);
            if (p < 0) p += h.box;
            k[d] = std::min(nc - 1, (int)(p / c.side));
        }
        key[I] = (k[0] * nc + k[1]) * nc + k[2];
    }
    c.start.assign((size_t)nc * nc * nc + 1, 0);
    for (int I = 0; I < N; ++I) c.start[key[I] + 1]++;
    for (size_t q = 1; q < c.start.size(); ++q) c.start[q] += c.start[q - 1];
    c.atoms.resize(N);
    std::vector<int> fill(c.start.begin(), c.start.end() - 1);
    for (int I = 0; I < N; ++I) c.atoms[fill[key[I]]++] = I;
    return c;
}

// Atoms within radius R of atom `centre` (minimum image), ascending.
void region_atoms(const HostMatrix& h, const Cells& cl, int centre, double R, std::vector<int>& out) {
    out.clear();
    const double cx = h.pos[3 * centre], cy = h.pos[3 * centre + 1], cz = h.pos[3 * centre + 2];
    const double R2 = R * R, box = h.box;
    auto test = [&](int I) {
        double dx = h.pos[3 * I] - cx, dy = h.pos[3 * I + 1] - cy, dz = h.pos[3 * I + 2] - cz;
        if (box > 0.0) {
            dx -= box * std::nearbyint(dx / box);
            dy -= box * std::nearbyint(dy / box);
            dz -= box * std::nearbyint(dz / box);
        }
        if (dx * dx + dy * dy + dz * dz <= R2) out.push_back(I);
    };
    const int reach = cl.nc > 0 ? (int)std::ceil(R / cl.side) : 0;
    if (cl.nc == 0 || 2 * reach + 1 >= cl.nc) {
        for (int I = 0; I < h.n_atoms; ++I) test(I);
        return;
    }
    const int nc = cl.nc;
    int k[3];
    for (int d = 0; d < 3; ++d) {
        double p = std::fmod(h.pos[3 * centre + d], box);
        if (p < 0) p += box;
        k[d] = std::min(nc - 1, (int)(p / cl.side));
    }
    for (int dx = -reach; dx <= reach; ++dx)
        for (int dy = -reach; dy <= reach; ++dy)
            for (int dz = -reach; dz <= reach; ++dz) {
                const int a = ((k[0] + dx) % nc + nc) % nc, b = ((k[1] + dy) % nc + nc) % nc,
                          c = ((k[2] + dz) % nc + nc) % nc;
                const int q = (a * nc + b) * nc + c;
                for (int t = cl.start[q]; t < cl.start[q + 1]; ++t) test(cl.atoms[t]);
            }
    std::sort(out.begin(), out.end());
}

void parallel_for(int n, const std::function<void(int, int)>& body) {
    int nt = (int)std::thread::hardware_concurrency();
    nt = std::max(1, std::min(nt, 32));
    nt = std::min(nt, std::max(1, n));
    std::atomic<int> next{0};
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            for (;;) {
                const int i = next.fetch_add(1);
                if (i >= n) break;
                body(i, t);
            }
        });
    for (auto& x : th) x.join();
}

struct RegionPlan {
    std::vector<int> atoms;   // ascending
    std::vector<int> row_len; // per local atom: nonzeros of each of its rows
    int m = 0, ncol = 0, cw = 1, nslice = 0;
    int64_t n_ent = 0, nnz = 0;
};

}  // namespace

const char* build_compact(const HostMatrix& h, int n_regions, const int* centres, const double* radii,
                          const uint8_t* orb_mask, bool want32, CompactHost& out) {
    const int N = h.n_atoms;
    out = CompactHost();
    const Cells cl = make_cells(h);
    std::vector<RegionPlan> plan(n_regions);
    int nthreads = std::max(1, std::min<int>((int)std::thread::hardware_concurrency(), 32));
    std::vector<std::vector<int>> loc_t(nthreads, std::vector<int>());
    std::atomic<int> too_big{0};
    // pass 1: members, row lengths, sizes
    parallel_for(n_regions, [&](int r, int t) {
        std::vector<int>& loc = loc_t[t];
        if (loc.empty()) loc.assign(N, -1);
        RegionPlan& P = plan[r];
        region_atoms(h, cl, centres[r], radii[r], P.atoms);
        for (size_t a = 0; a < P.atoms.size(); ++a) loc[P.atoms[a]] = (int)a;
        P.row_len.resize(P.atoms.size());
        int m = 0;
        int64_t ent = 0;
        for (size_t a = 0; a < P.atoms.size(); ++a) {
            const int I = P.atoms[a];
            int len = 0;
            for (int b = h.brow[I]; b < h.brow[I + 1]; ++b)
                if (loc[h.bcol[b]] >= 0) len += h.n_orb[h.bcol[b]];
            P.row_len[a] = len;
            m += h.n_orb[I];
            P.nnz += (int64_t)len * h.n_orb[I];
        }
        P.m = m;
        P.nslice = (m + 63) / 64;
        if (P.nslice * 64 > 65535) too_big.store(1);
        // rows sorted by length, longest first: slice lengths from the sorted rows
        std::vector<int> lens;
        lens.reserve(m);
        for (size_t a = 0; a < P.atoms.size(); ++a)
            for (int q = 0; q < h.n_orb[P.atoms[a]]; ++q) lens.push_back(P.row_len[a]);
        std::stable_sort(lens.begin(), lens.end(), std::greater<int>());
        for (int s = 0; s < P.nslice; ++s) ent += (int64_t)lens[64 * s] * 64;
        P.n_ent = ent;
        const int nI = h.n_orb[centres[r]];
        const int mask = (orb_mask && orb_mask[r]) ? (orb_mask[r] & ((1 << nI) - 1)) : ((1 << nI) - 1);
        P.ncol = __builtin_popcount(mask);
        P.cw = P.ncol <= 1 ? 1 : (P.ncol == 2 ? 2 : 4);
        for (int a : P.atoms) loc[a] = -1;
    });
    if (too_big.load()) return "a region holds more than 65535 orbitals";
    for (int r = 0; r < n_regions; ++r)
        if (plan[r].ncol == 0) return "a region has no columns (orbital mask selects nothing)";
    // offsets
    out.reg.resize(n_regions);
    int64_t ent = 0, pos = 0;
    int slice = 0, col = 0;
    std::vector<int64_t> pat0(n_regions);
    int64_t pat = 0;
    for (int r = 0; r < n_regions; ++r) {
        RegionDesc& D = out.reg[r];
        const RegionPlan& P = plan[r];
        D.m = P.m;
        D.nslice = P.nslice;
        D.slice0 = slice;
        D.col0 = col;
        D.ncol = P.ncol;
        D.cw = P.cw;
        D.ent0 = ent;
        D.pos0 = pos;
        pat0[r] = pat;
        ent += P.n_ent;
        pos += (int64_t)P.nslice * 64;
        slice += P.nslice;
        col += P.ncol;
        pat += (int64_t)P.ncol * h.atom_plen[centres[r]];
        out.max_slices = std::max(out.max_slices, P.nslice);
        out.lds_fp64 = std::max(out.lds_fp64, (size_t)P.nslice * 64 * P.cw * 8);
        out.lds_fp32 = std::max(out.lds_fp32, (size_t)P.nslice * 64 * P.cw * 4);
        out.region_orbs.push_back(P.m);
        out.region_nnz.push_back(P.nnz);
    }
    if (ent >= ((int64_t)1 << 40)) return "region layout too large";
    out.slice_len.assign(slice, 0);
    out.slice_ent.assign(slice, 0);
    out.idx.assign(ent, 0);
    const bool haveM = !h.M_in.empty();
    out.A64.assign(ent, 0.0);
    out.B64.assign(ent, 0.0);
    if (haveM) out.M64.assign(ent, 0.0);
    if (want32) {
        out.A32.assign(ent, 0.0f);
        out.B32.assign(ent, 0.0f);
        if (haveM) out.M32.assign(ent, 0.0f);
    }
    out.pos_row.assign(pos, 0xFFFF);
    out.cols.assign(col, 0);
    out.col_pos.assign(col, 0);
    out.col_region.assign(col, 0);
    out.pat_off.assign(col + 1, 0);
    out.pat_pos.assign(pat, -1);
    out.pat_B.assign(pat, 0.0);
    out.pat_A.assign(pat, 0.0);
    out.ritz_lo.assign(n_regions, 0.0);
    out.ritz_hi.assign(n_regions, 0.0);
    {
        int c = 0;
        for (int r = 0; r < n_regions; ++r)
            for (int q = 0; q < plan[r].ncol; ++q, ++c)
                out.pat_off[c + 1] = out.pat_off[c] + h.atom_plen[centres[r]];
    }
    std::atomic<int> bad{0};
    // half layout of B per region (mixed precision), concatenated after pass 2
    std::vector<std::vector<uint16_t>> hidx_r(want32 ? n_regions : 0);
    std::vector<std::vector<float>> hval_r(want32 ? n_regions : 0), hdiag_r(want32 ? n_regions : 0);
    std::vector<std::vector<int>> hlen_r(want32 ? n_regions : 0);
    std::vector<int> heb_r(n_regions, 0);
    out.region_hnnz.assign(n_regions, 0);
    // pass 2: layout of every region
    parallel_for(n_regions, [&](int r, int t) {
        std::vector<int>& loc = loc_t[t];
        if (loc.empty()) loc.assign(N, -1);
        const RegionPlan& P = plan[r];
        const RegionDesc& D = out.reg[r];
        const int na = (int)P.atoms.size();
        std::vector<int> aoff(na + 1, 0);
        for (int a = 0; a < na; ++a) {
            loc[P.atoms[a]] = a;
            aoff[a + 1] = aoff[a] + h.n_orb[P.atoms[a]];
        }
        // rows in order of decreasing length (stable): position -> row
        std::vector<int> row_atom(P.m), row_len(P.m), perm(P.m), row_pos(P.m);
        for (int a = 0; a < na; ++a)
            for (int q = aoff[a]; q < aoff[a + 1]; ++q) {
                row_atom[q] = a;
                row_len[q] = P.row_len[a];
            }
        for (int q = 0; q < P.m; ++q) perm[q] = q;
        std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return row_len[x] > row_len[y]; });
        for (int p = 0; p < P.m; ++p) row_pos[perm[p]] = p;
        for (int p = 0; p < P.m; ++p) out.pos_row[D.pos0 + p] = (uint16_t)perm[p];
        int64_t e_rel = 0;
        for (int s = 0; s < P.nslice; ++s) {
            const int len = row_len[perm[64 * s]];
            out.slice_len[D.slice0 + s] = len;
            out.slice_ent[D.slice0 + s] = (int)e_rel;
            for (int l = 0; l < 64; ++l) {
                const int p = 64 * s + l;
                int k = 0;
                const int64_t base = D.ent0 + e_rel + l;
                if (p < P.m) {
                    const int row = perm[p];
                    const int a = row_atom[row];
                    const int I = P.atoms[a];
                    const int al = row - aoff[a];
                    const int nI = h.n_orb[I];
                    for (int b = h.brow[I]; b < h.brow[I + 1]; ++b) {
                        const int J = h.bcol[b];
                        const int lj = loc[J];
                        if (lj < 0) continue;
                        const int nJ = h.n_orb[J];
                        const int64_t vo = h.in_voff[b] + (int64_t)al * nJ;
                        for (int be = 0; be < nJ; ++be, ++k) {
                            const int64_t e = base + (int64_t)k * 64;
                            out.idx[e] = (uint16_t)row_pos[aoff[lj] + be];
                            out.A64[e] = h.A_in[vo + be];
                            out.B64[e] = h.B_in[vo + be];
                            if (haveM) out.M64[e] = h.M_in[vo + be];
                            if (want32) {
                                out.A32[e] = (float)h.A_in[vo + be];
                                out.B32[e] = (float)h.B_in[vo + be];
                                if (haveM) out.M32[e] = (float)h.M_in[vo + be];
                            }
                        }
                    }
                    (void)nI;
                }
                if (k > len) bad.store(1);
                for (; k < len; ++k) out.idx[base + (int64_t)k * 64] = (uint16_t)p;  // zero padding
            }
            e_rel += (int64_t)len * 64;
        }
        if (e_rel != P.n_ent) bad.store(1);
        // half layout of B from the rows just laid out: each off-diagonal pair
        // {p, q} once, in row p when p + q is even and p < q or odd and p > q
        // (a balanced split: every row keeps about half its pairs), diagonal apart
        if (want32) {
            std::vector<int>& hl = hlen_r[r];
            std::vector<uint16_t>& hi = hidx_r[r];
            std::vector<float>& hv = hval_r[r];
            std::vector<float>& hd = hdiag_r[r];
            hl.assign(P.nslice, 0);
            hd.assign((size_t)P.nslice * 64, 0.0f);
            std::vector<std::vector<std::pair<uint16_t, float>>> lane_rows(64);
            std::vector<int> fan((size_t)P.nslice * 64, 0);  // transpose terms each position takes
            float bmax = 0.0f;
            int64_t stored = 0;
            for (int s = 0; s < P.nslice; ++s) {
                const int len = out.slice_len[D.slice0 + s];
                const int64_t e0 = D.ent0 + out.slice_ent[D.slice0 + s];
                int hmax = 0;
                for (int l = 0; l < 64; ++l) {
                    const int p = 64 * s + l;
                    auto& lr = lane_rows[l];
                    lr.clear();
                    const int real = p < P.m ? row_len[perm[p]] : 0;
                    for (int k = 0; k < real && k < len; ++k) {
                        const int64_t e = e0 + (int64_t)k * 64 + l;
                        const int q = out.idx[e];
                        const float b = out.B32[e];
                        if (q == p) {
                            hd[p] = b;
                        } else if (((p + q) & 1) == 0 ? (p < q) : (p > q)) {
                            lr.emplace_back((uint16_t)q, b);
                            bmax = std::max(bmax, std::fabs(b));
                            ++fan[q];
                        }
                    }
                    stored += (int64_t)lr.size();
                    hmax = std::max(hmax, (int)lr.size());
                }
                hl[s] = hmax;
                const size_t b0 = hi.size();
                hi.resize(b0 + (size_t)hmax * 64);
                hv.resize(b0 + (size_t)hmax * 64);
                for (int l = 0; l < 64; ++l) {
                    const int p = 64 * s + l;
                    const auto& lr = lane_rows[l];
                    for (int k = 0; k < hmax; ++k) {
                        const size_t e = b0 + (size_t)k * 64 + l;
                        hi[e] = k < (int)lr.size() ? lr[k].first : (uint16_t)p;  // zero padding
                        hv[e] = k < (int)lr.size() ? lr[k].second : 0.0f;
                    }
                }
            }
            int eb = 0;
            if (bmax > 0.0f) (void)std::frexp(bmax, &eb);  // bmax < 2^eb
            eb = std::max(eb, -60);                         // keeps the scaled x inside FP32 range
            const int fmax = *std::max_element(fan.begin(), fan.end());
            int L = 0;
            while ((1 << L) <= fmax) ++L;  // fmax < 2^L
            heb_r[r] = eb + L;
            out.region_hnnz[r] = stored;
        }
        // extreme Ritz values of the region's B: 40 Lanczos steps on the
        // layout just built (FP64 values), from a fixed pseudo-random start on
        // the region's rows (padding positions stay zero)
        {
            const int Pn = P.nslice * 64;
            std::vector<double> v(Pn, 0.0), vp(Pn, 0.0), w(Pn, 0.0);
            uint64_t xs = 0x9E3779B97F4A7C15ULL ^ ((uint64_t)(r + 1) * 0xD1B54A32D192ED03ULL);
            double nrm = 0.0;
            for (int p = 0; p < P.m; ++p) {
                xs ^= xs << 13;
                xs ^= xs >> 7;
                xs ^= xs << 17;
                v[p] = (double)(xs >> 11) / 9007199254740992.0 - 0.5;
                nrm += v[p] * v[p];
            }
            nrm = std::sqrt(nrm);
            for (int p = 0; p < P.m; ++p) v[p] /= nrm;
            auto bprod = [&](const std::vector<double>& x, std::vector<double>& y) {
                for (int s = 0; s < P.nslice; ++s) {
                    const int len = out.slice_len[D.slice0 + s];
                    const int64_t e0 = D.ent0 + out.slice_ent[D.slice0 + s];
                    for (int l = 0; l < 64; ++l) {
                        double acc = 0.0;
                        for (int k = 0; k < len; ++k) {
                            const int64_t e = e0 + (int64_t)k * 64 + l;
                            acc += out.B64[e] * x[out.idx[e]];
                        }
                        y[64 * s + l] = acc;
                    }
                }
            };
            std::vector<double> ta, tb;
            double bprev = 0.0;
            const int steps = std::min(P.m, 40);
            for (int k = 0; k < steps; ++k) {
                bprod(v, w);
                double al = 0.0;
                for (int p = 0; p < Pn; ++p) al += v[p] * w[p];
                double bb = 0.0;
                for (int p = 0; p < Pn; ++p) {
                    w[p] -= al * v[p] + bprev * vp[p];
                    bb += w[p] * w[p];
                }
                bb = std::sqrt(bb);
                ta.push_back(al);
                if (k + 1 == steps || !(bb > 1e-12 * std::fabs(al))) break;
                tb.push_back(bb);
                for (int p = 0; p < Pn; ++p) {
                    vp[p] = v[p];
                    v[p] = w[p] / bb;
                }
                bprev = bb;
            }
            tb.resize(ta.size() - 1);
            out.ritz_lo[r] = tri_eig(ta, tb, 0);
            out.ritz_hi[r] = tri_eig(ta, tb, (int)ta.size() - 1);
        }
        // columns and their patterns (the caller's pattern of column j: the
        // orbitals of the atoms coupled to j's atom, ascending)
        const int C = centres[r];
        const int nC = h.n_orb[C];
        const int mask = (orb_mask && orb_mask[r]) ? (orb_mask[r] & ((1 << nC) - 1)) : ((1 << nC) - 1);
        int c = D.col0;
        int64_t po = pat0[r];
        for (int q = 0; q < nC; ++q) {
            if (!((mask >> q) & 1)) continue;
            out.cols[c] = h.atom_off[C] + q;
            out.col_pos[c] = row_pos[aoff[loc[C]] + q];
            out.col_region[c] = r;
            for (int b = h.brow[C]; b < h.brow[C + 1]; ++b) {
                const int J = h.bcol[b];
                const int nJ = h.n_orb[J];
                const int lj = loc[J];
                for (int be = 0; be < nJ; ++be, ++po) {
                    out.pat_pos[po] = lj >= 0 ? row_pos[aoff[lj] + be] : -1;
                    out.pat_B[po] = h.B_in[h.in_voff[b] + (int64_t)q * nJ + be];
                    out.pat_A[po] = h.A_in[h.in_voff[b] + (int64_t)q * nJ + be];
                }
            }
            ++c;
        }
        for (int a : P.atoms) loc[a] = -1;
    });
    if (bad.load()) return "internal: region layout sizes disagree";
    if (want32) {
        int64_t he = 0;
        out.hslice_len.assign(out.slice_len.size(), 0);
        out.hslice_ent.assign(out.slice_len.size(), 0);
        for (int r = 0; r < n_regions; ++r) {
            RegionDesc& D = out.reg[r];
            D.hent0 = he;
            D.heb = heb_r[r];
            int64_t rel = 0;
            for (int s = 0; s < D.nslice; ++s) {
                out.hslice_len[D.slice0 + s] = hlen_r[r][s];
                out.hslice_ent[D.slice0 + s] = (int)rel;
                rel += (int64_t)hlen_r[r][s] * 64;
            }
            he += rel;
        }
        out.hidx.resize(he);
        out.hval.resize(he);
        out.hdiag.assign(out.pos_row.size(), 0.0f);
        parallel_for(n_regions, [&](int r, int) {
            const RegionDesc& D = out.reg[r];
            std::copy(hidx_r[r].begin(), hidx_r[r].end(), out.hidx.begin() + D.hent0);
            std::copy(hval_r[r].begin(), hval_r[r].end(), out.hval.begin() + D.hent0);
            std::copy(hdiag_r[r].begin(), hdiag_r[r].end(), out.hdiag.begin() + D.pos0);
            std::vector<uint16_t>().swap(hidx_r[r]);
            std::vector<float>().swap(hval_r[r]);
            std::vector<float>().swap(hdiag_r[r]);
        });
    }
    for (int r = 0; r < n_regions; ++r) out.useful += (int64_t)plan[r].m * plan[r].ncol;
    return nullptr;
}

}  // namespace elses
