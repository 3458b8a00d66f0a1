// C ABI of the gfx950 generalized shifted Krylov solver: argument checks,
// upload of the atom-block matrices, the spectral bracket of B, and the
// host loop that drives the fused passes.
//
// Solver structure (paper Sec. III: (zB - A) x = e_j for many z, Eqs. 9, 13, 14):
//  * A B-inner-product Lanczos process for B^{-1}A started from B^{-1} e_j
//    spans the shift-invariant Krylov space K_n(B^{-1}A; B^{-1}e_j), shared by
//    every shift; its vectors are real.
//  * Each Lanczos step needs one overlap solve v = B^{-1} s.  It is done with a
//    fixed-degree Richardson iteration whose step lengths are the Chebyshev
//    roots of an interval enclosing the spectrum of B.  Being a fixed
//    polynomial p(B), the process is the exact Lanczos process of the pencil
//    (A, p(B)^{-1}); the degree is chosen so that ||I - p(B) B|| <= inner_tol.
//    The solve runs on s = s' - alpha_n t_n itself (alpha_n is reduced between
//    the A pass and the first overlap step), which keeps q = p(B) t to
//    rounding at every step.
//  * A block of `ld` columns ("slots") advances together; every pass is one
//    sparse product with the block plus the step's element-wise work.  When
//    a column has converged for all shifts its slot takes the next column.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace elses {
void launch_lanczos_orth(double* w, const double* v, const double* u, double a, double b, int n, hipStream_t st);
void launch_lanczos_shift(double* u, double* v, const double* w, double s, int n, hipStream_t st);
// Smallest / largest eigenvalue of the symmetric tridiagonal (a, b) by
// Sturm-sequence bisection.
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
    int cnt = 0;
    double d = 1.0;
    for (size_t i = 0; i < a.size(); ++i) {
        const double bb = (i == 0) ? 0.0 : b[i - 1] * b[i - 1];
        d = (a[i] - x) - (i == 0 ? 0.0 : bb / d);
        if (d == 0.0) d = -1e-300;
        if (d < 0) ++cnt;
    }
    return cnt;
}

double tri_eig(const std::vector<double>& a, const std::vector<double>& b, int idx) {
    double lo = 1e300, hi = -1e300;
    for (size_t i = 0; i < a.size(); ++i) {
        const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < a.size() ? fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (sturm_count(a, b, mid) > idx)
            hi = mid;
        else
            lo = mid;
    }
    return 0.5 * (lo + hi);
}

}  // namespace elses

using namespace elses;

namespace {

struct HipFail {
    hipError_t e;
    const char* what;
};

#define HCHECK(call)                                 \
    do {                                             \
        hipError_t _e = (call);                      \
        if (_e != hipSuccess) throw HipFail{_e, #call}; \
    } while (0)

elses_status set_err(elses_ctx ctx, elses_status s, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return s;
}

template <typename T>
T* dalloc(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) throw HipFail{e, "hipMalloc"};
    return static_cast<T*>(p);
}

// RAII list of device allocations of one call
struct DevPool {
    std::vector<void*> ptrs;
    template <typename T>
    T* get(size_t n) {
        T* p = dalloc<T>(n);
        ptrs.push_back(p);
        return p;
    }
    ~DevPool() {
        for (void* p : ptrs) (void)hipFree(p);
    }
};

// Clusters of at most max_atoms consecutive atoms whose coupled orbitals
// (the union over the cluster) fit in max_rows LDS rows.  Greedy in atom
// order.  bloc[b] (internal block order) receives the LDS row of block b's
// first coupled orbital.  Returns false if a single atom couples to more
// orbitals than the LDS holds (then this cluster shape is not used).
bool build_clusters(int max_atoms, int max_rows, const std::vector<int>& atom_off, const std::vector<int>& brow,
                    const std::vector<int>& bcol, const std::vector<int>& borb, std::vector<int>& cl_atom,
                    std::vector<int>& cl_uoff, std::vector<int>& cl_urow, std::vector<int>& bloc) {
    const int N = (int)atom_off.size() - 1;
    std::vector<int> stamp(N, -1), lrow(N, 0);
    cl_atom.assign(1, 0);
    cl_uoff.assign(1, 0);
    cl_urow.clear();
    bloc.assign(bcol.size(), 0);
    int I = 0, c = 0;
    std::vector<int> members;
    while (I < N) {
        int orbs = 0;
        const int start = I;
        members.clear();
        while (I < N && I - start < max_atoms) {
            int add = 0;
            for (int b = brow[I]; b < brow[I + 1]; ++b)
                if (stamp[bcol[b]] != c) add += atom_off[bcol[b] + 1] - atom_off[bcol[b]];
            if (orbs + add > max_rows) {
                if (I == start) return false;
                break;
            }
            for (int b = brow[I]; b < brow[I + 1]; ++b)
                if (stamp[bcol[b]] != c) {
                    stamp[bcol[b]] = c;
                    members.push_back(bcol[b]);
                }
            orbs += add;
            ++I;
        }
        std::sort(members.begin(), members.end());
        int r = 0;
        for (int J : members) {
            lrow[J] = r;
            for (int q = atom_off[J]; q < atom_off[J + 1]; ++q, ++r) cl_urow.push_back(q);
        }
        // borb holds the first orbital of the coupled atom in internal order
        for (int A = start; A < I; ++A)
            for (int b = brow[A]; b < brow[A + 1]; ++b) {
                const int o = borb[b];
                // map orbital -> atom via the members (atom_off is ascending)
                const int J = (int)(std::upper_bound(atom_off.begin(), atom_off.end(), o) - atom_off.begin()) - 1;
                bloc[b] = lrow[J];
            }
        cl_atom.push_back(I);
        cl_uoff.push_back((int)cl_urow.size());
        ++c;
    }
    return true;
}

// Row groups for the grouped passes.  Every 1-orbital atom joins the
// 4-orbital atom it couples to most strongly through B (the sum of |B| over
// the block; the overlap decays with distance, so this is its nearest
// 4-orbital neighbour), at most kGroupH per 4-orbital atom; the others stay
// alone.  Groups are emitted in atom order (a 4-orbital atom's group at its
// own position).  The union of a group's coupled atoms is listed 4-orbital
// atoms first (ascending), then 1-orbital ones; the values are dense
// R x n_J blocks over it, in the same order, zero where a member does not
// couple to the union atom.
struct HostGroups {
    std::vector<int> R, roff{0}, rows, uoff{0}, u4, uorb;
    std::vector<int64_t> voff;
    std::vector<double> A, B;
};

void build_groups(const elses_system* sys, const HostMatrix& h, const std::vector<int64_t>& in_voff,
                  HostGroups& G) {
    const int N = h.n_atoms;
    const int8_t* no = sys->n_orb;
    struct Cand {
        double w;
        int hh, J;
    };
    std::vector<Cand> cand;
    for (int a = 0; a < N; ++a) {
        if (no[a] != 1) continue;
        for (int b = h.brow[a]; b < h.brow[a + 1]; ++b) {
            const int J = h.bcol[b];
            if (no[J] != 4) continue;
            double w = 0.0;
            for (int q = 0; q < 4; ++q) w += fabs(sys->B_val[in_voff[b] + q]);
            cand.push_back({w, a, J});
        }
    }
    std::sort(cand.begin(), cand.end(), [](const Cand& x, const Cand& y) {
        if (x.w != y.w) return x.w > y.w;
        if (x.hh != y.hh) return x.hh < y.hh;
        return x.J < y.J;
    });
    std::vector<int> owner(N, -1), cnt(N, 0);
    for (const Cand& c : cand)
        if (owner[c.hh] < 0 && cnt[c.J] < kGroupH) {
            owner[c.hh] = c.J;
            ++cnt[c.J];
        }
    std::vector<std::vector<int>> attached(N);
    for (int a = 0; a < N; ++a)
        if (owner[a] >= 0) attached[owner[a]].push_back(a);  // ascending by construction
    std::vector<int> stamp(N, -1), upos(N, 0), members, u4list, u1list;
    int g = 0;
    for (int I = 0; I < N; ++I) {
        if (no[I] == 1 && owner[I] >= 0) continue;
        members.assign(1, I);
        if (no[I] == 4) members.insert(members.end(), attached[I].begin(), attached[I].end());
        int R = 0;
        for (int m : members) {
            for (int q = 0; q < no[m]; ++q) G.rows.push_back(h.atom_off[m] + q);
            R += no[m];
        }
        u4list.clear();
        u1list.clear();
        for (int m : members)
            for (int b = h.brow[m]; b < h.brow[m + 1]; ++b) {
                const int J = h.bcol[b];
                if (stamp[J] == g) continue;
                stamp[J] = g;
                (no[J] == 4 ? u4list : u1list).push_back(J);
            }
        std::sort(u4list.begin(), u4list.end());
        std::sort(u1list.begin(), u1list.end());
        const int n4u = (int)u4list.size();
        for (int k = 0; k < n4u; ++k) upos[u4list[k]] = k;
        for (int k = 0; k < (int)u1list.size(); ++k) upos[u1list[k]] = n4u + k;
        const int64_t base = (int64_t)G.A.size();
        const int64_t len = (int64_t)R * (4 * n4u + (int64_t)u1list.size());
        G.A.resize(base + len, 0.0);
        G.B.resize(base + len, 0.0);
        int rm = 0;
        for (int m : members) {
            for (int b = h.brow[m]; b < h.brow[m + 1]; ++b) {
                const int J = h.bcol[b];
                const int nJ = no[J];
                const int k = upos[J];
                const int64_t off = base + (k < n4u ? (int64_t)k * R * 4 : (int64_t)n4u * R * 4 + (int64_t)(k - n4u) * R);
                for (int al = 0; al < no[m]; ++al)
                    for (int be = 0; be < nJ; ++be) {
                        const int64_t dst = off + (int64_t)(rm + al) * nJ + be;
                        G.A[dst] = sys->A_val[in_voff[b] + al * nJ + be];
                        G.B[dst] = sys->B_val[in_voff[b] + al * nJ + be];
                    }
            }
            rm += no[m];
        }
        for (int J : u4list) G.uorb.push_back(h.atom_off[J]);
        for (int J : u1list) G.uorb.push_back(h.atom_off[J]);
        G.R.push_back(R);
        G.roff.push_back((int)G.rows.size());
        G.u4.push_back(G.uoff.back() + n4u);
        G.uoff.push_back((int)G.uorb.size());
        G.voff.push_back(base);
        ++g;
    }
}

}  // namespace

namespace elses {

// Richardson iteration for B v = s with the d roots of the Chebyshev
// polynomial of the interval [lo, hi] as inverse step lengths,
//   x_1 = s / theta_0,  x_{k+1} = x_k + (s - B x_k) / theta_k,
// so the residual after d-1 products is prod_k (1 - B/theta_k) s, the scaled
// Chebyshev polynomial T_d((c - B)/h) / T_d(c/h) with c = (hi+lo)/2,
// h = (hi-lo)/2.  The roots are taken in Leja order, which keeps the
// intermediate residuals bounded.  d is the smallest degree with
// 1/T_d(c/h) <= tol.
Rich richardson_plan(double lo, double hi, double tol) {
    Rich r;
    const double cen = 0.5 * (hi + lo), half = 0.5 * (hi - lo);
    const double sigma = cen / half;
    double t0 = 1.0, t1 = sigma;
    int d = 1;
    while (1.0 / t1 > tol && d < kRichMaxDegree) {
        const double t2 = 2.0 * sigma * t1 - t0;
        t0 = t1;
        t1 = t2;
        ++d;
    }
    r.d = std::max(d, 3);  // a first step, at least one middle or last step
    r.reached = 1.0 / t1;
    const double pi = 3.14159265358979323846;
    std::vector<double> roots(r.d);
    for (int i = 0; i < r.d; ++i) roots[i] = cen + half * cos((2.0 * i + 1.0) * pi / (2.0 * r.d));
    std::vector<double> ord;
    std::vector<char> used(r.d, 0);
    int first = 0;
    for (int i = 1; i < r.d; ++i)
        if (fabs(roots[i]) > fabs(roots[first])) first = i;
    used[first] = 1;
    ord.push_back(roots[first]);
    for (int k = 1; k < r.d; ++k) {
        int best = -1;
        double bv = -1.0;
        for (int i = 0; i < r.d; ++i) {
            if (used[i]) continue;
            double p = 0.0;  // log of the product of distances
            for (double o : ord) p += log(fabs(roots[i] - o));
            if (best < 0 || p > bv) {
                bv = p;
                best = i;
            }
        }
        used[best] = 1;
        ord.push_back(roots[best]);
    }
    r.g0 = 1.0 / ord[0];
    for (int k = 1; k < r.d; ++k) r.tau.push_back(1.0 / ord[k]);
    return r;
}

}  // namespace elses

namespace {

// A plan capped at kRichMaxDegree steps does not reach its tolerance: the
// overlap solve would be less accurate than asked.  Refuse such solves.
elses_status check_rich(elses_ctx ctx, const Rich& r, double tol, double lo, double hi) {
    if (r.reached <= tol * (1.0 + 1e-12)) return ELSES_OK;
    return set_err(ctx, ELSES_ERR_INVALID_ARG,
                   "the overlap solve on B's interval [" + std::to_string(lo) + ", " + std::to_string(hi) +
                       "] would need more than " + std::to_string(kRichMaxDegree) +
                       " Richardson steps to reach " + std::to_string(tol) + " (it reaches " +
                       std::to_string(r.reached) + ")");
}

}  // namespace

// Scratch of the allocation-free region solve (elses_regions_solve_noalloc):
// a file-scope device array that every GPU the library runs on holds until
// the process ends.  In host code its name is only a stand-in; the device
// address of each GPU's copy is taken once per device at context creation.
constexpr size_t kNoAllocBytes = (size_t)256 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

extern "C" {

const char* elses_version(void) { return "elses-gfx950 0.3"; }

void elses_opts_default(elses_opts* o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->tol = 1e-8;
    o->max_outer = 20000;
    o->inner_tol = 1e-13;
    o->out_mode = ELSES_OUT_PATTERN;
    o->slots = 0;
    o->use_mixed = 0;
    o->audit = 0;
    o->inner_max = 200;
}

elses_status elses_ctx_create(int device, void* hip_stream, elses_ctx* out) {
    if (!out) return ELSES_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return ELSES_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return ELSES_ERR_HIP;
    // this device's address of the allocation-free entry point's scratch array
    if (device >= kMaxDevices) return ELSES_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            void* p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ELSES_ERR_HIP;
            g_scratch_ptr[device] = p;
        }
    }
    auto* c = new elses_ctx_s();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
    *out = c;
    return ELSES_OK;
}

void elses_ctx_destroy(elses_ctx ctx) { delete ctx; }

const char* elses_last_error(elses_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void elses_mat_destroy(elses_mat m) {
    if (!m) return;
    DevMatrix& d = m->d;
    void* ptrs[] = {d.atom_off, d.orb_atom, d.brow, d.bsplit, d.borb, d.voff, d.asc_borb,
                    d.asc_n,    d.asc_voff, d.A,    d.B,      d.A32,  d.B32, m->M_dev};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (auto& C : d.cl) {
        void* q[] = {C.atom, C.uoff, C.urow, C.bloc};
        for (void* p : q)
            if (p) (void)hipFree(p);
    }
    {
        auto& D = d.grp;
        void* q[] = {D.R, D.roff, D.rows, D.uoff, D.u4, D.uorb, D.voff, D.A, D.B, D.A32, D.B32};
        for (void* p : q)
            if (p) (void)hipFree(p);
    }
    delete m;
}

}  // extern "C"

namespace {

// Matrix creation.  bracket == nullptr: a caller's matrix (kept on the host
// too, for carving regions; spectral bracket of B by Lanczos).  Otherwise an
// internal batched matrix whose B spectrum lies inside the given interval.
elses_status mat_create_impl(elses_ctx ctx, const elses_system* sys, int precision, const double* bracket,
                             elses_mat* out) {
    if (!ctx) return ELSES_ERR_INVALID_ARG;
    if (!out || !sys) return set_err(ctx, ELSES_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    const int N = sys->n_atoms;
    if (N <= 0 || !sys->n_orb || !sys->blk_row_ptr || !sys->blk_col || !sys->A_val || !sys->B_val)
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "empty system or null array");
    if (precision != ELSES_FP64 && precision != ELSES_MIXED)
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "precision must be ELSES_FP64 or ELSES_MIXED");
    HostMatrix h;
    h.n_atoms = N;
    h.atom_off.assign(N + 1, 0);
    for (int I = 0; I < N; ++I) {
        const int no = sys->n_orb[I];
        if (no != 1 && no != 4) return set_err(ctx, ELSES_ERR_INVALID_ARG, "n_orb must be 1 or 4");
        h.atom_off[I + 1] = h.atom_off[I] + no;
    }
    const int64_t Mll = h.atom_off[N];
    if (Mll >= (int64_t)1 << 30) return set_err(ctx, ELSES_ERR_INVALID_ARG, "too many orbitals");
    h.M = (int)Mll;
    const int64_t* rp = sys->blk_row_ptr;
    if (rp[0] != 0) return set_err(ctx, ELSES_ERR_INVALID_ARG, "blk_row_ptr[0] must be 0");
    for (int I = 0; I < N; ++I)
        if (rp[I + 1] <= rp[I]) return set_err(ctx, ELSES_ERR_INVALID_ARG, "every block row needs its diagonal");
    const int64_t nnzb = rp[N];
    if (nnzb >= (int64_t)1 << 31) return set_err(ctx, ELSES_ERR_INVALID_ARG, "too many blocks");
    h.brow.assign(N + 1, 0);
    h.bcol.assign(nnzb, 0);
    h.atom_plen.assign(N, 0);
    std::vector<int64_t> in_voff(nnzb + 1, 0);  // caller's value offset of each block
    int64_t vo = 0;
    for (int I = 0; I < N; ++I) {
        h.brow[I] = (int)rp[I];
        const int nI = sys->n_orb[I];
        bool diag = false;
        int plen = 0;
        for (int64_t b = rp[I]; b < rp[I + 1]; ++b) {
            const int J = sys->blk_col[b];
            if (J < 0 || J >= N) return set_err(ctx, ELSES_ERR_INVALID_ARG, "blk_col out of range");
            if (b > rp[I] && J <= sys->blk_col[b - 1])
                return set_err(ctx, ELSES_ERR_INVALID_ARG, "blk_col must be strictly ascending in a row");
            if (J == I) diag = true;
            h.bcol[b] = J;
            in_voff[b] = vo;
            vo += (int64_t)nI * sys->n_orb[J];
            plen += sys->n_orb[J];
        }
        if (!diag) return set_err(ctx, ELSES_ERR_INVALID_ARG, "missing diagonal block");
        h.atom_plen[I] = plen;
        h.pmax = std::max(h.pmax, plen);
    }
    h.brow[N] = (int)nnzb;
    in_voff[nnzb] = vo;
    const int64_t nnz = vo;
    // Internal layout: per row, the 4-orbital neighbours first, then the
    // 1-orbital ones (each ascending); values re-laid out in that order.
    std::vector<int> bsplit(N), borb(nnzb), asc_borb(nnzb), asc_n(nnzb);
    std::vector<int64_t> voff(N), asc_voff(nnzb), perm_voff(nnzb);  // perm_voff: internal offset of block b
    {
        int64_t o = 0;
        for (int I = 0; I < N; ++I) {
            const int nI = sys->n_orb[I];
            voff[I] = o;
            int pos = h.brow[I];
            for (int pass = 0; pass < 2; ++pass) {
                const int want = pass == 0 ? 4 : 1;
                if (pass == 1) bsplit[I] = pos;
                for (int b = h.brow[I]; b < h.brow[I + 1]; ++b) {
                    const int J = h.bcol[b];
                    if (sys->n_orb[J] != want) continue;
                    borb[pos++] = h.atom_off[J];
                    perm_voff[b] = o;
                    o += (int64_t)nI * want;
                }
            }
        }
        for (int b = 0; b < (int)nnzb; ++b) {
            asc_borb[b] = h.atom_off[h.bcol[b]];
            asc_n[b] = sys->n_orb[h.bcol[b]];
            asc_voff[b] = perm_voff[b];
        }
    }
    // symmetry of pattern and values, finiteness
    for (int I = 0; I < N; ++I) {
        const int nI = sys->n_orb[I];
        for (int b = h.brow[I]; b < h.brow[I + 1]; ++b) {
            const int J = h.bcol[b];
            const int nJ = sys->n_orb[J];
            const int* beg = h.bcol.data() + h.brow[J];
            const int* end = h.bcol.data() + h.brow[J + 1];
            const int* f = std::lower_bound(beg, end, I);
            if (f == end || *f != I) return set_err(ctx, ELSES_ERR_INVALID_ARG, "block pattern is not symmetric");
            const int64_t bt = (int64_t)(f - h.bcol.data());
            for (int x = 0; x < nI; ++x)
                for (int y = 0; y < nJ; ++y) {
                    const double a1 = sys->A_val[in_voff[b] + x * nJ + y];
                    const double a2 = sys->A_val[in_voff[bt] + y * nI + x];
                    const double b1 = sys->B_val[in_voff[b] + x * nJ + y];
                    const double b2 = sys->B_val[in_voff[bt] + y * nI + x];
                    if (!std::isfinite(a1) || !std::isfinite(b1))
                        return set_err(ctx, ELSES_ERR_INVALID_ARG, "non-finite matrix value");
                    if (a1 != a2 || b1 != b2) return set_err(ctx, ELSES_ERR_INVALID_ARG, "A or B not symmetric");
                }
        }
    }
    if (sys->pos) h.pos.assign(sys->pos, sys->pos + 3 * (size_t)N);
    h.box = sys->box;
    if (!bracket) {
        h.n_orb.assign(sys->n_orb, sys->n_orb + N);
        h.in_voff = in_voff;
        h.A_in.assign(sys->A_val, sys->A_val + nnz);
        h.B_in.assign(sys->B_val, sys->B_val + nnz);
    }

    auto* m = new elses_mat_s();
    m->ctx = ctx;
    m->precision = precision;
    DevMatrix& d = m->d;
    d.n_atoms = N;
    d.M = h.M;
    d.nnzb = (int)nnzb;
    d.nnz = nnz;
    try {
        HCHECK(hipSetDevice(ctx->device));
        std::vector<int> orb_atom(h.M);
        for (int I = 0; I < N; ++I)
            for (int q = h.atom_off[I]; q < h.atom_off[I + 1]; ++q) orb_atom[q] = I;
        // values in the internal block order
        std::vector<double> Ai(nnz), Bi(nnz);
        for (int I = 0; I < N; ++I)
            for (int b = h.brow[I]; b < h.brow[I + 1]; ++b) {
                const int64_t len = (int64_t)sys->n_orb[I] * sys->n_orb[h.bcol[b]];
                std::copy(sys->A_val + in_voff[b], sys->A_val + in_voff[b] + len, Ai.begin() + perm_voff[b]);
                std::copy(sys->B_val + in_voff[b], sys->B_val + in_voff[b] + len, Bi.begin() + perm_voff[b]);
            }
        d.atom_off = dalloc<int>(N + 1);
        d.orb_atom = dalloc<int>(h.M);
        d.brow = dalloc<int>(N + 1);
        d.bsplit = dalloc<int>(N);
        d.borb = dalloc<int>(nnzb);
        d.voff = dalloc<int64_t>(N);
        d.asc_borb = dalloc<int>(nnzb);
        d.asc_n = dalloc<int>(nnzb);
        d.asc_voff = dalloc<int64_t>(nnzb);
        d.A = dalloc<double>(nnz);
        d.B = dalloc<double>(nnz);
        HCHECK(hipMemcpy(d.atom_off, h.atom_off.data(), sizeof(int) * (N + 1), hipMemcpyHostToDevice));
        HCHECK(hipMemcpy(d.orb_atom, orb_atom.data(), sizeof(int) * h.M, hipMemcpyHostToDevice));
        HCHECK(hipMemcpy(d.brow, h.brow.data(), sizeof(int) * (N + 1), hipMemcpyHostToDevice));
        HCHECK(hipMemcpy(d.bsplit, bsplit.data(), sizeof(int) * N, hipMemcpyHostToDevice));
        HCHECK(hipMemcpy(d.borb, borb.data(), sizeof(int) * nnzb, hipMemcpyHostToDevice));
        HCHECK(hipMemcpy(d.voff, voff.data(), sizeof(int64_t) * N, hipMemcpyHostToDevice));
        HCHECK(hipMemcpy(d.asc_borb, asc_borb.data(), sizeof(int) * nnzb, hipMemcpyHostToDevice));
        HCHECK(hipMemcpy(d.asc_n, asc_n.data(), sizeof(int) * nnzb, hipMemcpyHostToDevice));
        HCHECK(hipMemcpy(d.asc_voff, asc_voff.data(), sizeof(int64_t) * nnzb, hipMemcpyHostToDevice));
        {
            HostGroups G;
            build_groups(sys, h, in_voff, G);
            h.grp_row0.resize(G.R.size());  // moved into m->h below
            for (size_t g = 0; g < G.R.size(); ++g) h.grp_row0[g] = G.rows[G.roff[g]];
            auto& D = d.grp;
            D.n = (int)G.R.size();
            D.nval = (int64_t)G.A.size();
            D.R = dalloc<int>(G.R.size());
            D.roff = dalloc<int>(G.roff.size());
            D.rows = dalloc<int>(G.rows.size());
            D.uoff = dalloc<int>(G.uoff.size());
            D.u4 = dalloc<int>(G.u4.size());
            D.uorb = dalloc<int>(G.uorb.size());
            D.voff = dalloc<int64_t>(G.voff.size());
            D.A = dalloc<double>(G.A.size());
            D.B = dalloc<double>(G.B.size());
            HCHECK(hipMemcpy(D.R, G.R.data(), sizeof(int) * G.R.size(), hipMemcpyHostToDevice));
            HCHECK(hipMemcpy(D.roff, G.roff.data(), sizeof(int) * G.roff.size(), hipMemcpyHostToDevice));
            HCHECK(hipMemcpy(D.rows, G.rows.data(), sizeof(int) * G.rows.size(), hipMemcpyHostToDevice));
            HCHECK(hipMemcpy(D.uoff, G.uoff.data(), sizeof(int) * G.uoff.size(), hipMemcpyHostToDevice));
            HCHECK(hipMemcpy(D.u4, G.u4.data(), sizeof(int) * G.u4.size(), hipMemcpyHostToDevice));
            HCHECK(hipMemcpy(D.uorb, G.uorb.data(), sizeof(int) * G.uorb.size(), hipMemcpyHostToDevice));
            HCHECK(hipMemcpy(D.voff, G.voff.data(), sizeof(int64_t) * G.voff.size(), hipMemcpyHostToDevice));
            HCHECK(hipMemcpy(D.A, G.A.data(), sizeof(double) * G.A.size(), hipMemcpyHostToDevice));
            HCHECK(hipMemcpy(D.B, G.B.data(), sizeof(double) * G.B.size(), hipMemcpyHostToDevice));
            if (precision == ELSES_MIXED) {
                std::vector<float> t(G.A.size());
                D.A32 = dalloc<float>(G.A.size());
                D.B32 = dalloc<float>(G.B.size());
                for (size_t i = 0; i < t.size(); ++i) t[i] = (float)G.A[i];
                HCHECK(hipMemcpy(D.A32, t.data(), sizeof(float) * t.size(), hipMemcpyHostToDevice));
                for (size_t i = 0; i < t.size(); ++i) t[i] = (float)G.B[i];
                HCHECK(hipMemcpy(D.B32, t.data(), sizeof(float) * t.size(), hipMemcpyHostToDevice));
            }
        }
        for (int sh = 0; sh < kStageShapes; ++sh) {
            std::vector<int> cl_atom, cl_uoff, cl_urow, bloc;
            if (build_clusters(kStageWaves[sh], kStageRows[sh], h.atom_off, h.brow, h.bcol, borb, cl_atom, cl_uoff,
                               cl_urow, bloc)) {
                DevMatrix::Clusters& C = d.cl[sh];
                C.n = (int)cl_atom.size() - 1;
                C.atom = dalloc<int>(cl_atom.size());
                C.uoff = dalloc<int>(cl_uoff.size());
                C.urow = dalloc<int>(cl_urow.size());
                C.bloc = dalloc<int>(bloc.size());
                HCHECK(hipMemcpy(C.atom, cl_atom.data(), sizeof(int) * cl_atom.size(), hipMemcpyHostToDevice));
                HCHECK(hipMemcpy(C.uoff, cl_uoff.data(), sizeof(int) * cl_uoff.size(), hipMemcpyHostToDevice));
                HCHECK(hipMemcpy(C.urow, cl_urow.data(), sizeof(int) * cl_urow.size(), hipMemcpyHostToDevice));
                HCHECK(hipMemcpy(C.bloc, bloc.data(), sizeof(int) * bloc.size(), hipMemcpyHostToDevice));
            }
        }
        HCHECK(hipMemcpy(d.A, Ai.data(), sizeof(double) * nnz, hipMemcpyHostToDevice));
        HCHECK(hipMemcpy(d.B, Bi.data(), sizeof(double) * nnz, hipMemcpyHostToDevice));
        if (precision == ELSES_MIXED) {
            std::vector<float> t(nnz);
            d.A32 = dalloc<float>(nnz);
            d.B32 = dalloc<float>(nnz);
            for (int64_t i = 0; i < nnz; ++i) t[i] = (float)Ai[i];
            HCHECK(hipMemcpy(d.A32, t.data(), sizeof(float) * nnz, hipMemcpyHostToDevice));
            for (int64_t i = 0; i < nnz; ++i) t[i] = (float)Bi[i];
            HCHECK(hipMemcpy(d.B32, t.data(), sizeof(float) * nnz, hipMemcpyHostToDevice));
        }
        m->h = std::move(h);

        if (bracket) {
            m->b_lo = bracket[0];
            m->b_hi = bracket[1];
        } else {
            // Spectral bracket of B: Lanczos sweep from a fixed pseudo-random start.
            const int M = d.M;
            const int steps = std::min(M, 80);
            hipStream_t st = ctx->stream;
            DevPool pool;
            double* v = pool.get<double>(M);
            double* u = pool.get<double>(M);
            double* w = pool.get<double>(M);
            const int nbl = std::min(256, (M + 255) / 256);
            double* part = pool.get<double>(nbl);
            std::vector<double> hv(M), hp(nbl);
            uint64_t s = 0x2545F4914F6CDD1DULL;
            double nrm = 0;
            for (int i = 0; i < M; ++i) {
                s ^= s << 13;
                s ^= s >> 7;
                s ^= s << 17;
                hv[i] = (double)(s >> 11) / 9007199254740992.0 - 0.5;
                nrm += hv[i] * hv[i];
            }
            nrm = sqrt(nrm);
            for (int i = 0; i < M; ++i) hv[i] /= nrm;
            HCHECK(hipMemcpyAsync(v, hv.data(), sizeof(double) * M, hipMemcpyHostToDevice, st));
            HCHECK(hipMemsetAsync(u, 0, sizeof(double) * M, st));
            std::vector<double> ta, tb;
            double bprev = 0.0;
            auto dotdev = [&](const double* x, const double* y) {
                launch_dot_partial(x, y, M, part, nbl, st);
                HCHECK(hipMemcpyAsync(hp.data(), part, sizeof(double) * nbl, hipMemcpyDeviceToHost, st));
                HCHECK(hipStreamSynchronize(st));
                double acc = 0;
                for (double q : hp) acc += q;
                return acc;
            };
            for (int k = 0; k < steps; ++k) {
                launch_spmm_generic(d, d.B, 1, 1, v, w, st);
                const double al = dotdev(v, w);
                launch_lanczos_orth(w, v, u, al, bprev, M, st);
                ta.push_back(al);
                const double bb = sqrt(std::max(dotdev(w, w), 0.0));
                if (k + 1 == steps || bb <= 1e-12 * fabs(al)) break;
                tb.push_back(bb);
                launch_lanczos_shift(u, v, w, 1.0 / bb, M, st);
                bprev = bb;
            }
            HCHECK(hipGetLastError());
            tb.resize(ta.size() > 0 ? ta.size() - 1 : 0);
            const double tmin = tri_eig(ta, tb, 0);
            const double tmax = tri_eig(ta, tb, (int)ta.size() - 1);
            const double width = tmax - tmin;
            m->b_lo = tmin - 0.02 * width - 1e-3 * fabs(tmin);
            m->b_hi = tmax + 0.02 * width + 1e-3 * fabs(tmax);
            if (!(m->b_lo > 0.0) || !std::isfinite(m->b_hi)) {
                char buf[160];
                snprintf(buf, sizeof buf, "overlap B is not positive definite (Lanczos bracket [%g, %g])", tmin, tmax);
                elses_mat_destroy(m);
                return set_err(ctx, ELSES_ERR_NOT_SPD, buf);
            }
        }
    } catch (const HipFail& f) {
        elses_mat_destroy(m);
        const elses_status s = (f.e == hipErrorOutOfMemory) ? ELSES_ERR_OOM : ELSES_ERR_HIP;
        return set_err(ctx, s, std::string(f.what) + ": " + hipGetErrorString(f.e));
    }
    *out = m;
    return ELSES_OK;
}

}  // namespace

extern "C" {

elses_status elses_mat_create(elses_ctx ctx, const elses_system* sys, int precision, elses_mat* out) {
    return mat_create_impl(ctx, sys, precision, nullptr, out);
}

elses_status elses_mat_info(elses_mat m, int64_t* M, int64_t* pmax, double* b_lo, double* b_hi) {
    if (!m) return ELSES_ERR_INVALID_ARG;
    if (M) *M = m->d.M;
    if (pmax) *pmax = m->h.pmax;
    if (b_lo) *b_lo = m->b_lo;
    if (b_hi) *b_hi = m->b_hi;
    return ELSES_OK;
}

elses_status elses_pattern(elses_mat m, int32_t n_cols, const int32_t* cols, int64_t* pat_off, int32_t* rows) {
    if (!m) return ELSES_ERR_INVALID_ARG;
    elses_ctx ctx = m->ctx;
    if (n_cols < 0 || (n_cols > 0 && !cols) || !pat_off) return set_err(ctx, ELSES_ERR_INVALID_ARG, "bad arguments");
    const HostMatrix& h = m->h;
    std::vector<int> orb_atom(h.M);
    for (int I = 0; I < h.n_atoms; ++I)
        for (int q = h.atom_off[I]; q < h.atom_off[I + 1]; ++q) orb_atom[q] = I;
    pat_off[0] = 0;
    for (int c = 0; c < n_cols; ++c) {
        if (cols[c] < 0 || cols[c] >= h.M) return set_err(ctx, ELSES_ERR_INVALID_ARG, "column out of range");
        const int J = orb_atom[cols[c]];
        pat_off[c + 1] = pat_off[c] + h.atom_plen[J];
        if (rows) {
            int64_t o = pat_off[c];
            for (int b = h.brow[J]; b < h.brow[J + 1]; ++b) {
                const int I = h.bcol[b];
                for (int q = h.atom_off[I]; q < h.atom_off[I + 1]; ++q) rows[o++] = q;
            }
        }
    }
    return ELSES_OK;
}

}  // extern "C"

namespace {

// Fill the matrix and layout fields of `pa` for the sparse-pass variant
// (0 auto = grouped with 4 waves per group, 1 direct, 2/3 LDS-staged cluster
// shape 0/1, 4/5/6 grouped with 4/2/1 waves per group) and block count ld (a
// multiple of 64).  Returns an error message or null.
const char* configure_pass(const DevMatrix& d, int variant_in, int ld, PassArgs& pa) {
    if (ld <= 0 || ld % 64 != 0) return "column block must be a multiple of 64";
    // bits 4-5 select the workgroup placement, bit 6 forces one column per
    // lane, bit 7 limits the FP32 passes to two columns per lane
    const int variant = variant_in & 15;
    pa.place = (variant_in >> 4) & 3;
    const bool force_cpl1 = (variant_in >> 6) & 1;
    const bool cap32 = (variant_in >> 7) & 1;
    int mode, split = 4;
    if (variant == 0) {
        // measured best on MI355X for the hydrocarbon pencils: row groups split
        // over two waves, XCD regions walked tile-fastest
        mode = d.grp.n > 0 ? 9 : 0;
        split = 2;
        if (variant_in == 0) pa.place = 1;
    } else if (variant == 1) {
        mode = 0;
    } else if (variant >= 2 && variant < 2 + kStageShapes) {
        if (d.cl[variant - 2].n == 0) return "LDS-staged passes unavailable for this matrix";
        mode = variant - 1;
    } else if (variant >= 2 + kStageShapes && variant <= 4 + kStageShapes) {
        if (d.grp.n == 0) return "grouped passes unavailable for this matrix";
        mode = 9;
        split = 4 >> (variant - 2 - kStageShapes);
    } else {
        return "variant must be 0 (auto), 1 (direct), 2/3 (LDS-staged) or 4/5/6 (grouped)";
    }
    pa.group_split = split;
    pa.atom_off = d.atom_off;
    pa.brow = d.brow;
    pa.bsplit = d.bsplit;
    pa.borb = d.borb;
    pa.voff = d.voff;
    pa.n_atoms = d.n_atoms;
    pa.ld = ld;
    pa.staged = mode;
    pa.atoms_per_slab = kWavesPerBlock;
    const bool cluster = (mode == 1 || mode == 2);
    const int cpl = (cluster || force_cpl1) ? 1 : ((ld % 128 == 0) ? 2 : 1);
    pa.n_tiles = ld / (64 * cpl);
    const int cpl32 = (cluster || force_cpl1) ? 1 : ((ld % 256 == 0 && !cap32) ? 4 : ((ld % 128 == 0) ? 2 : 1));
    pa.n_tiles32 = ld / (64 * cpl32);
    // the column split needs the tile count to be a multiple of 8 or to divide 8
    auto splits = [](int t) { return t % 8 == 0 || 8 % t == 0; };
    if (pa.place == 3 && (!splits(pa.n_tiles) || !splits(pa.n_tiles32))) pa.place = 1;
    if (cluster) {
        const auto& C = d.cl[mode - 1];
        pa.n_clusters = C.n;
        pa.cl_atom = C.atom;
        pa.cl_uoff = C.uoff;
        pa.cl_urow = C.urow;
        pa.bloc = C.bloc;
        pa.n_slabs = ((C.n + 7) / 8) * 8;
    } else if (mode == 9) {
        pa.n_grp = d.grp.n;
        pa.g_R = d.grp.R;
        pa.g_roff = d.grp.roff;
        pa.g_rows = d.grp.rows;
        pa.g_uoff = d.grp.uoff;
        pa.g_u4 = d.grp.u4;
        pa.g_uorb = d.grp.uorb;
        pa.g_voff = d.grp.voff;
        const int gpw = kWavesPerBlock / split;  // groups per workgroup
        pa.n_slabs = (((d.grp.n + gpw - 1) / gpw + 7) / 8) * 8;
    } else {
        pa.n_slabs = (((d.n_atoms + kWavesPerBlock - 1) / kWavesPerBlock + 7) / 8) * 8;
    }
    return nullptr;
}

int choose_slots(int n_cols, int M, const elses_opts& o) {
    if (o.slots > 0) return o.slots;
    int ld = ((n_cols + 63) / 64) * 64;
    // keep the five working blocks of [M][ld] doubles within ~1.5 GiB and ld <= 1024
    // (per-column cost of the passes is lowest near 1024 columns on MI355X; wider
    // blocks overflow the 256 MB last-level cache)
    const int64_t cap_mem = (int64_t)(1.5 * 1024 * 1024 * 1024) / (5 * 8 * (int64_t)std::max(M, 1));
    int cap = (int)std::min<int64_t>(1024, std::max<int64_t>(64, (cap_mem / 64) * 64));
    ld = std::min(ld, cap);
    if (ld > 128 && ld % 128 != 0 && ld + 64 <= cap) ld += 64;
    return std::max(ld, 64);
}

}  // namespace

// Region problems packed into tiles of one block-diagonal matrix.  A region
// is the principal sub-pencil of the atoms within a radius of a centre atom
// (the paper's real-space projection, Sec. III-B); its columns are the
// centre atom's orbitals.  Consecutive regions fill tiles of L column slots;
// tile t's block holds the union of its regions' atoms, and a per-(row,
// column) bit marks the rows inside each column's own region.  Keeping every
// vector zero outside its region makes each column's solve exactly that of
// its region's sub-pencil, while all columns of a tile share one pass over
// the union.
struct elses_regions_s {
    elses_ctx ctx = nullptr;
    elses_mat gm = nullptr;  // the caller's matrix (not owned)
    elses_mat bm = nullptr;  // block-diagonal tile matrix (owned; tile layout only)
    int L = 64, n_tiles = 0, n_cols = 0, n_regions = 0;
    // compact layout (tile_width 0): every region on its own, one persistent launch
    bool compact = false;
    struct Compact {
        std::vector<RegionDesc> reg;
        std::vector<int> col_region, region_nnz, order;
        std::vector<int64_t> region_ent;
        std::vector<double> ritz_lo, ritz_hi;  // extreme Ritz values of each region's B
        // regions grouped by vector width (4, 2, 1): group g is order[goff[g] .. goff[g+1]);
        // one launch per group
        int goff[4] = {0, 0, 0, 0};
        int gcw[3] = {4, 2, 1};
        int gmaxP[3] = {0, 0, 0};
        int64_t lane_rows = 0;  // sum over regions of positions x column width
        bool has32 = false;
        RegionDesc* d_reg = nullptr;
        int *d_order = nullptr, *d_slice_len = nullptr, *d_slice_ent = nullptr, *d_col_pos = nullptr,
            *d_pat_pos = nullptr;
        uint16_t *d_idx = nullptr, *d_pos_row = nullptr;
        double *d_A64 = nullptr, *d_B64 = nullptr, *d_pat_B = nullptr, *d_pat_A = nullptr, *d_M64 = nullptr;
        float *d_A32 = nullptr, *d_B32 = nullptr, *d_M32 = nullptr;
        int64_t* d_pat_off = nullptr;
        bool hasM = false;  // the learned preconditioner was carved with the regions
        // half layout of B (mixed precision): stored off-diagonal pairs per region
        std::vector<int64_t> region_hnnz;
        int *d_hslice_len = nullptr, *d_hslice_ent = nullptr;
        uint16_t* d_hidx = nullptr;
        float *d_hval = nullptr, *d_hdiag = nullptr;
    } cp;
    std::vector<int> cols;         // global orbital of each column, region by region
    std::vector<int> col_row;      // row of each column's unit vector in bm
    std::vector<int> slot_map;     // [n_tiles * L] column of each slot or -1
    std::vector<int64_t> pat_off;  // [n_cols + 1] offsets of the global pattern of each column
    std::vector<int> rows;         // bm row of each pattern entry, -1 outside the region
    std::vector<int64_t> vidx;     // internal value index of X_ji in gm per pattern entry
    std::vector<int> group_tile;   // tile of each row group of bm (non-decreasing)
    std::vector<int> region_orbs;  // orbitals of each region
    std::vector<int> centres;      // centre atom of each region
    std::vector<int> region_tile;
    std::vector<int> tile_row0;    // [n_tiles + 1] first row of each tile in bm
    int64_t useful = 0;            // sum over columns of their region's orbitals
    uint64_t* d_mask = nullptr;
    int* d_col_row = nullptr;
    int* d_rows = nullptr;
    int64_t* d_vidx = nullptr;
    int64_t* d_pat_off = nullptr;
    int* d_slot_map = nullptr;
    int* d_row_tile = nullptr;  // tile of each row of bm
    ~elses_regions_s() {
        void* p[] = {d_mask, d_col_row, d_rows, d_vidx, d_pat_off, d_slot_map, d_row_tile};
        for (void* q : p)
            if (q) (void)hipFree(q);
        void* c[] = {cp.d_reg,   cp.d_order, cp.d_slice_len, cp.d_slice_ent, cp.d_col_pos, cp.d_pat_pos,
                     cp.d_idx,   cp.d_pos_row, cp.d_A64,     cp.d_B64,       cp.d_pat_B,   cp.d_pat_A,
                     cp.d_A32,   cp.d_B32,   cp.d_pat_off,   cp.d_M64,       cp.d_M32,
                     cp.d_hslice_len, cp.d_hslice_ent, cp.d_hidx, cp.d_hval, cp.d_hdiag};
        for (void* q : c)
            if (q) (void)hipFree(q);
        if (bm) elses_mat_destroy(bm);
    }
};

namespace {

template <typename T>
T* upload(const std::vector<T>& v) {
    T* p = dalloc<T>(v.size());
    if (!v.empty()) HCHECK(hipMemcpy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return p;
}

// Compact layout: each region's principal sub-pencil laid out on its own
// (region.hip), solved by one persistent launch with a costliest-first queue.
elses_status compact_create_impl(elses_ctx ctx, elses_mat gm, int n_regions, const int32_t* centres,
                                 const double* radii, const uint8_t* orb_mask, elses_regions* out) {
    const HostMatrix& h = gm->h;
    CompactHost H;
    const char* err = build_compact(h, n_regions, centres, radii, orb_mask, gm->precision == ELSES_MIXED, H);
    if (err) return set_err(ctx, ELSES_ERR_INVALID_ARG, err);
    if (H.max_slices * 64 > 8192)
        return set_err(ctx, ELSES_ERR_INVALID_ARG,
                       "a region exceeds 8192 orbitals, the compact layout's limit; use tile_width 64 or 128");
    auto* P = new elses_regions_s();
    P->centres.assign(centres, centres + n_regions);
    P->ctx = ctx;
    P->gm = gm;
    P->L = 0;
    P->compact = true;
    P->n_regions = n_regions;
    P->n_tiles = 0;
    P->cols = H.cols;
    P->pat_off = H.pat_off;
    P->region_orbs = H.region_orbs;
    P->n_cols = (int)H.cols.size();
    P->useful = H.useful;
    auto& C = P->cp;
    C.reg = H.reg;
    C.col_region = H.col_region;
    C.ritz_lo = H.ritz_lo;
    C.ritz_hi = H.ritz_hi;
    C.has32 = gm->precision == ELSES_MIXED;
    // per region: nonzeros (algorithmic bytes) and padded entries; lane-rows
    C.region_nnz.assign(n_regions, 0);
    C.region_ent.assign(n_regions, 0);
    for (int r = 0; r < n_regions; ++r) {
        const RegionDesc& D = H.reg[r];
        C.region_nnz[r] = (int)H.region_nnz[r];
        C.region_ent[r] = (r + 1 < n_regions ? H.reg[r + 1].ent0 : (int64_t)H.idx.size()) - D.ent0;
        C.lane_rows += (int64_t)D.nslice * 64 * D.cw;
    }
    // queue order per vector width: costliest region first, the cost of a
    // region outer step taken as nonzeros x sqrt(kappa of its B overlap
    // interval), the growth of the Chebyshev-Richardson degree
    std::vector<double> cost(n_regions, 0.0);
    for (int r = 0; r < n_regions; ++r) {
        const double tl = H.ritz_lo[r], th = H.ritz_hi[r], w = th - tl;
        const double lo = std::max(gm->b_lo, tl - 0.02 * w - 1e-3 * std::fabs(tl));
        const double hi = std::min(gm->b_hi, th + 0.02 * w + 1e-3 * std::fabs(th));
        cost[r] = (double)H.region_nnz[r] * std::sqrt(hi / std::max(lo, 1e-300));
    }
    C.order.clear();
    for (int g = 0; g < 3; ++g) {
        C.goff[g] = (int)C.order.size();
        std::vector<int> grp;
        for (int r = 0; r < n_regions; ++r)
            if (H.reg[r].cw == C.gcw[g]) {
                grp.push_back(r);
                C.gmaxP[g] = std::max(C.gmaxP[g], H.reg[r].nslice * 64);
            }
        std::stable_sort(grp.begin(), grp.end(), [&](int a, int b) { return cost[a] > cost[b]; });
        C.order.insert(C.order.end(), grp.begin(), grp.end());
    }
    C.goff[3] = (int)C.order.size();
    try {
        C.d_reg = upload(H.reg);
        C.d_order = upload(C.order);
        C.d_slice_len = upload(H.slice_len);
        C.d_slice_ent = upload(H.slice_ent);
        C.d_col_pos = upload(H.col_pos);
        C.d_pat_pos = upload(H.pat_pos);
        C.d_idx = upload(H.idx);
        C.d_pos_row = upload(H.pos_row);
        C.d_A64 = upload(H.A64);
        C.d_B64 = upload(H.B64);
        C.d_pat_B = upload(H.pat_B);
        C.d_pat_A = upload(H.pat_A);
        C.d_pat_off = upload(H.pat_off);
        if (C.has32) {
            C.d_A32 = upload(H.A32);
            C.d_B32 = upload(H.B32);
            C.d_hslice_len = upload(H.hslice_len);
            C.d_hslice_ent = upload(H.hslice_ent);
            C.d_hidx = upload(H.hidx);
            C.d_hval = upload(H.hval);
            C.d_hdiag = upload(H.hdiag);
            C.region_hnnz = H.region_hnnz;
        }
        if (!H.M64.empty()) {
            C.hasM = true;
            C.d_M64 = upload(H.M64);
            if (C.has32) C.d_M32 = upload(H.M32);
        }
    } catch (const HipFail& f) {
        delete P;
        const elses_status s = (f.e == hipErrorOutOfMemory) ? ELSES_ERR_OOM : ELSES_ERR_HIP;
        return set_err(ctx, s, std::string(f.what) + ": " + hipGetErrorString(f.e));
    }
    *out = P;
    return ELSES_OK;
}

elses_status regions_check(elses_ctx ctx, elses_mat gm, int n_regions, const int32_t* centres, const double* radii) {
    const HostMatrix& h = gm->h;
    const int N = h.n_atoms;
    if (h.n_orb.empty()) return set_err(ctx, ELSES_ERR_INVALID_ARG, "regions need a caller-created matrix");
    if (h.pos.empty()) return set_err(ctx, ELSES_ERR_INVALID_ARG, "regions need atom positions (pos)");
    if (n_regions < 1 || !centres || !radii) return set_err(ctx, ELSES_ERR_INVALID_ARG, "no regions");
    std::vector<char> seen(N, 0);
    for (int r = 0; r < n_regions; ++r) {
        if (centres[r] < 0 || centres[r] >= N) return set_err(ctx, ELSES_ERR_INVALID_ARG, "centre out of range");
        if (seen[centres[r]]) return set_err(ctx, ELSES_ERR_INVALID_ARG, "duplicate centre");
        seen[centres[r]] = 1;
        if (!(radii[r] > 0.0) || !std::isfinite(radii[r]))
            return set_err(ctx, ELSES_ERR_INVALID_ARG, "radii must be finite and > 0");
    }
    return ELSES_OK;
}

elses_status regions_create_impl(elses_ctx ctx, elses_mat gm, int n_regions, const int32_t* centres,
                                 const double* radii, const uint8_t* orb_mask, int tile_width, elses_regions* out) {
    const HostMatrix& h = gm->h;
    const int N = h.n_atoms;
    {
        const elses_status st = regions_check(ctx, gm, n_regions, centres, radii);
        if (st != ELSES_OK) return st;
    }
    if (tile_width == 0) return compact_create_impl(ctx, gm, n_regions, centres, radii, orb_mask, out);
    // orbitals of each centre solved as columns
    std::vector<int> cmask(n_regions);
    for (int r = 0; r < n_regions; ++r) {
        const int all = (1 << h.n_orb[centres[r]]) - 1;
        cmask[r] = (orb_mask && orb_mask[r]) ? (orb_mask[r] & all) : all;
        if (cmask[r] == 0) return set_err(ctx, ELSES_ERR_INVALID_ARG, "a region has no columns (orbital mask selects nothing)");
    }
    const int L = tile_width;
    if (L != 64 && L != 128) return set_err(ctx, ELSES_ERR_INVALID_ARG, "tile_width must be 0, 64 or 128");
    auto* P = new elses_regions_s();
    P->centres.assign(centres, centres + n_regions);
    P->ctx = ctx;
    P->gm = gm;
    P->L = L;
    P->n_regions = n_regions;
    // region membership: minimum-image distance to the centre <= radius
    const double box = h.box;
    std::vector<std::vector<int>> reg(n_regions);
    for (int r = 0; r < n_regions; ++r) {
        const int c = centres[r];
        const double cx = h.pos[3 * c], cy = h.pos[3 * c + 1], cz = h.pos[3 * c + 2];
        const double R2 = radii[r] * radii[r];
        int orbs = 0;
        for (int I = 0; I < N; ++I) {
            double dx = h.pos[3 * I] - cx, dy = h.pos[3 * I + 1] - cy, dz = h.pos[3 * I + 2] - cz;
            if (box > 0.0) {
                dx -= box * std::nearbyint(dx / box);
                dy -= box * std::nearbyint(dy / box);
                dz -= box * std::nearbyint(dz / box);
            }
            if (dx * dx + dy * dy + dz * dz <= R2) {
                reg[r].push_back(I);
                orbs += h.n_orb[I];
            }
        }
        P->region_orbs.push_back(orbs);
    }
    // tiles: consecutive regions while their columns fit
    std::vector<int> tile_r0{0};
    {
        int used = 0;
        for (int r = 0; r < n_regions; ++r) {
            const int nc = __builtin_popcount(cmask[r]);
            if (used + nc > L) {
                tile_r0.push_back(r);
                used = 0;
            }
            used += nc;
        }
        tile_r0.push_back(n_regions);
    }
    const int T = (int)tile_r0.size() - 1;
    P->n_tiles = T;
    P->slot_map.assign((size_t)T * L, -1);
    // block-diagonal system of the tile unions
    std::vector<int8_t> bn_orb;
    std::vector<int64_t> brp{0};
    std::vector<int32_t> bcol;
    std::vector<double> bA, bB;
    std::vector<int> stamp(N, -1), loc(N, -1);
    std::vector<int> tile_row0, tile_atom0;
    std::vector<std::vector<int>> tile_atoms(T);
    int atom_base = 0, row_base = 0;
    for (int t = 0; t < T; ++t) {
        std::vector<int>& U = tile_atoms[t];
        for (int r = tile_r0[t]; r < tile_r0[t + 1]; ++r)
            for (int I : reg[r])
                if (stamp[I] != t) {
                    stamp[I] = t;
                    U.push_back(I);
                }
        std::sort(U.begin(), U.end());
        for (size_t k = 0; k < U.size(); ++k) loc[U[k]] = atom_base + (int)k;
        tile_atom0.push_back(atom_base);
        tile_row0.push_back(row_base);
        for (int I : U) {
            bn_orb.push_back(h.n_orb[I]);
            const int nI = h.n_orb[I];
            for (int b = h.brow[I]; b < h.brow[I + 1]; ++b) {
                const int J = h.bcol[b];
                if (stamp[J] != t) continue;
                bcol.push_back(loc[J]);
                const int64_t len = (int64_t)nI * h.n_orb[J];
                bA.insert(bA.end(), h.A_in.begin() + h.in_voff[b], h.A_in.begin() + h.in_voff[b] + len);
                bB.insert(bB.end(), h.B_in.begin() + h.in_voff[b], h.B_in.begin() + h.in_voff[b] + len);
            }
            brp.push_back((int64_t)bcol.size());
            row_base += nI;
        }
        atom_base += (int)U.size();
    }
    tile_atom0.push_back(atom_base);
    tile_row0.push_back(row_base);
    P->tile_row0 = tile_row0;
    elses_system bsys{};
    bsys.n_atoms = atom_base;
    bsys.n_orb = bn_orb.data();
    bsys.blk_row_ptr = brp.data();
    bsys.blk_col = bcol.data();
    bsys.A_val = bA.data();
    bsys.B_val = bB.data();
    bsys.pos = nullptr;
    bsys.box = 0.0;
    const double bracket[2] = {gm->b_lo, gm->b_hi};  // principal submatrices: Cauchy interlacing
    elses_status st = mat_create_impl(ctx, &bsys, gm->precision, bracket, &P->bm);
    if (st != ELSES_OK) {
        delete P;
        return st;
    }
    const int Mb = P->bm->d.M;
    std::vector<int> brow_off(atom_base + 1, 0);
    for (int a = 0; a < atom_base; ++a) brow_off[a + 1] = brow_off[a] + bn_orb[a];
    // columns, slots, masks, patterns
    const int mw = L / 64;
    std::vector<uint64_t> mask((size_t)Mb * mw, 0);
    std::vector<int64_t> asc_voff(h.brow[N]);
    try {
        HCHECK(hipMemcpy(asc_voff.data(), gm->d.asc_voff, sizeof(int64_t) * asc_voff.size(), hipMemcpyDeviceToHost));
    } catch (const HipFail& f) {
        delete P;
        return set_err(ctx, ELSES_ERR_HIP, std::string(f.what) + ": " + hipGetErrorString(f.e));
    }
    P->pat_off.push_back(0);
    for (int t = 0; t < T; ++t) {
        for (int k = 0; k < (int)tile_atoms[t].size(); ++k) loc[tile_atoms[t][k]] = tile_atom0[t] + k;
        int slot = 0;
        for (int r = tile_r0[t]; r < tile_r0[t + 1]; ++r) {
            P->region_tile.push_back(t);
            const int C = centres[r];
            std::vector<char> inreg;  // membership of the tile's union atoms
            inreg.assign(tile_atoms[t].size(), 0);
            for (int I : reg[r]) inreg[loc[I] - tile_atom0[t]] = 1;
            const int c_first = (int)P->cols.size();
            for (int q = 0; q < h.n_orb[C]; ++q) {
                if (!((cmask[r] >> q) & 1)) continue;
                const int cidx = (int)P->cols.size();
                P->cp.col_region.push_back(r);
                P->cols.push_back(h.atom_off[C] + q);
                P->col_row.push_back(brow_off[loc[C]] + q);
                P->slot_map[(size_t)t * L + slot] = cidx;
                for (int I : reg[r])
                    for (int row = brow_off[loc[I]]; row < brow_off[loc[I] + 1]; ++row)
                        mask[(size_t)row * mw + (slot >> 6)] |= 1ull << (slot & 63);
                ++slot;
                P->useful += P->region_orbs[r];
                // pattern of column (C, q) in the caller's matrix
                for (int b = h.brow[C]; b < h.brow[C + 1]; ++b) {
                    const int J = h.bcol[b];
                    const int nJ = h.n_orb[J];
                    const bool inside = stamp[J] >= 0 && loc[J] >= tile_atom0[t] && loc[J] < tile_atom0[t + 1] &&
                                        inreg[loc[J] - tile_atom0[t]];
                    for (int al = 0; al < nJ; ++al) {
                        P->rows.push_back(inside ? brow_off[loc[J]] + al : -1);
                        P->vidx.push_back(asc_voff[b] + (int64_t)q * nJ + al);
                    }
                }
                P->pat_off.push_back((int64_t)P->rows.size());
            }
            (void)c_first;
        }
    }
    P->n_cols = (int)P->cols.size();
    // tile of each row and of each row group
    std::vector<int> row_tile(Mb);
    {
        for (int t = 0; t < T; ++t)
            for (int row = tile_row0[t]; row < tile_row0[t + 1]; ++row) row_tile[row] = t;
        P->group_tile.resize(P->bm->h.grp_row0.size());
        for (size_t g = 0; g < P->group_tile.size(); ++g) P->group_tile[g] = row_tile[P->bm->h.grp_row0[g]];
        for (size_t g = 1; g < P->group_tile.size(); ++g)
            if (P->group_tile[g] < P->group_tile[g - 1]) {
                delete P;
                return set_err(ctx, ELSES_ERR_HIP, "internal: row groups are not ordered by tile");
            }
    }
    try {
        P->d_mask = dalloc<uint64_t>(mask.size());
        P->d_col_row = dalloc<int>(P->col_row.size());
        P->d_rows = dalloc<int>(P->rows.size());
        P->d_vidx = dalloc<int64_t>(P->vidx.size());
        P->d_pat_off = dalloc<int64_t>(P->pat_off.size());
        P->d_slot_map = dalloc<int>(P->slot_map.size());
        P->d_row_tile = dalloc<int>(row_tile.size());
        HCHECK(hipMemcpy(P->d_row_tile, row_tile.data(), sizeof(int) * row_tile.size(), hipMemcpyHostToDevice));
        HCHECK(hipMemcpy(P->d_mask, mask.data(), sizeof(uint64_t) * mask.size(), hipMemcpyHostToDevice));
        HCHECK(hipMemcpy(P->d_col_row, P->col_row.data(), sizeof(int) * P->col_row.size(), hipMemcpyHostToDevice));
        HCHECK(hipMemcpy(P->d_rows, P->rows.data(), sizeof(int) * P->rows.size(), hipMemcpyHostToDevice));
        HCHECK(hipMemcpy(P->d_vidx, P->vidx.data(), sizeof(int64_t) * P->vidx.size(), hipMemcpyHostToDevice));
        HCHECK(hipMemcpy(P->d_pat_off, P->pat_off.data(), sizeof(int64_t) * P->pat_off.size(),
                         hipMemcpyHostToDevice));
        HCHECK(hipMemcpy(P->d_slot_map, P->slot_map.data(), sizeof(int) * P->slot_map.size(),
                         hipMemcpyHostToDevice));
    } catch (const HipFail& f) {
        delete P;
        const elses_status s = (f.e == hipErrorOutOfMemory) ? ELSES_ERR_OOM : ELSES_ERR_HIP;
        return set_err(ctx, s, std::string(f.what) + ": " + hipGetErrorString(f.e));
    }
    *out = P;
    return ELSES_OK;
}

// Slab tables of the grouped passes over region tiles: every slab holds row
// groups of one tile; chunks of up to 64 slabs of one tile feed the per-tile
// reductions.  Sets the slab count, mask and tile fields of pa.
const char* region_slabs(const elses_regions_s* rp, PassArgs& pa, std::vector<int>& slab_group,
                         std::vector<int>& slab_tile, std::vector<int>& chunk_s0, std::vector<int>& chunk_s1,
                         std::vector<int>& tile_chunk_off) {
    if (pa.staged != 9) return "region solves use the grouped passes";
    const int gpw = kWavesPerBlock / pa.group_split;
    const int ng = (int)rp->group_tile.size();
    if (ng == 0) return "region tiles have no row groups";
    tile_chunk_off.push_back(0);
    int g = 0;
    for (int t = 0; t < rp->n_tiles; ++t) {
        const int g0 = g;
        while (g < ng && rp->group_tile[g] == t) ++g;
        const int s0 = (int)slab_tile.size();
        for (int q = g0; q < g; q += gpw) {
            for (int i = 0; i < gpw; ++i) slab_group.push_back(q + i < g ? q + i : -1);
            slab_tile.push_back(t);
        }
        const int s1 = (int)slab_tile.size();
        for (int q = s0; q < s1; q += 64) {
            chunk_s0.push_back(q);
            chunk_s1.push_back(std::min(q + 64, s1));
        }
        tile_chunk_off.push_back((int)chunk_s0.size());
    }
    while (slab_tile.size() % 8 != 0) {
        for (int i = 0; i < gpw; ++i) slab_group.push_back(-1);
        slab_tile.push_back(0);
    }
    pa.n_slabs = (int)slab_tile.size();
    pa.n_tiles = pa.n_tiles32 = 1;
    pa.mask_words = rp->L / 64;
    pa.mask = rp->d_mask;
    return nullptr;
}

elses_status solve_core(elses_ctx ctx, elses_mat mat, int n_cols, const int32_t* cols, int K,
                        const double* shifts, const double* cw, const elses_opts* opts_in, double* x_out,
                        int32_t* iters_out, double* resid_out, double* rho_out, double* traces_out,
                        double* col_traces_out, const elses_regions_s* rp = nullptr) {
    if (!ctx || !mat) return ELSES_ERR_INVALID_ARG;
    elses_opts o;
    elses_opts_default(&o);
    if (opts_in) o = *opts_in;
    // gd: the caller's matrix (columns, patterns, trace values); d: the
    // matrix of the passes (gd, or the block-diagonal region tiles)
    const DevMatrix& gd = mat->d;
    const DevMatrix& d = rp ? rp->bm->d : mat->d;
    const HostMatrix& h = mat->h;
    const int M = d.M;
    const bool density = (cw != nullptr);
    if (n_cols < 0) return set_err(ctx, ELSES_ERR_INVALID_ARG, "n_cols < 0");
    if (K < 1 || K > 256) return set_err(ctx, ELSES_ERR_INVALID_ARG, "n_shifts must be in [1, 256]");
    if (!shifts) return set_err(ctx, ELSES_ERR_INVALID_ARG, "shifts is null");
    for (int k = 0; k < K; ++k) {
        if (!std::isfinite(shifts[2 * k]) || !std::isfinite(shifts[2 * k + 1]) || !(shifts[2 * k + 1] > 0.0))
            return set_err(ctx, ELSES_ERR_INVALID_ARG, "every shift needs a finite value with Im z > 0");
        if (density && (!std::isfinite(cw[2 * k]) || !std::isfinite(cw[2 * k + 1])))
            return set_err(ctx, ELSES_ERR_INVALID_ARG, "non-finite density weight");
    }
    if (!(o.tol > 0.0) || !std::isfinite(o.tol)) return set_err(ctx, ELSES_ERR_INVALID_ARG, "tol must be > 0");
    if (o.max_outer < 1) return set_err(ctx, ELSES_ERR_INVALID_ARG, "max_outer must be >= 1");
    if (!(o.inner_tol > 0.0 && o.inner_tol < 1.0))
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "inner_tol must be in (0, 1)");
    if (o.out_mode != ELSES_OUT_PATTERN && o.out_mode != ELSES_OUT_FULL)
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "out_mode must be PATTERN or FULL");
    if (o.slots < 0 || o.slots % 64 != 0 || o.slots > 65536)
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "slots must be 0 or a multiple of 64 up to 65536");
    if (o.use_mixed && mat->precision != ELSES_MIXED)
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "use_mixed needs a matrix created with ELSES_MIXED");
    const bool full = (o.out_mode == ELSES_OUT_FULL);
    if (o.audit && (!full || !x_out || !resid_out))
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "audit needs ELSES_OUT_FULL with x_out and resid_out");
    if (density && full) return set_err(ctx, ELSES_ERR_INVALID_ARG, "density matrix output uses the pattern mode");
    if (n_cols > 0 && !cols) return set_err(ctx, ELSES_ERR_INVALID_ARG, "cols is null");
    if (rp && full) return set_err(ctx, ELSES_ERR_INVALID_ARG, "region solves use the pattern mode");
    if (!rp) {
        std::vector<char> seen(M, 0);
        for (int c = 0; c < n_cols; ++c) {
            if (cols[c] < 0 || cols[c] >= M) return set_err(ctx, ELSES_ERR_INVALID_ARG, "column out of range");
            if (seen[cols[c]]) return set_err(ctx, ELSES_ERR_INVALID_ARG, "duplicate column");
            seen[cols[c]] = 1;
        }
    }
    const bool want_pre = o.precond != 0;
    if (want_pre) {
        if (rp)
            return set_err(ctx, ELSES_ERR_INVALID_ARG,
                           "the learned preconditioner runs in global solves and compact region sets, not in tiles");
        if (o.use_mixed)
            return set_err(ctx, ELSES_ERR_INVALID_ARG, "the preconditioned global solve runs in FP64 (use_mixed = 0)");
        if (o.graph)
            return set_err(ctx, ELSES_ERR_INVALID_ARG, "graph replay is not available with the preconditioned solve");
        if (!mat->M_dev)
            return set_err(ctx, ELSES_ERR_INVALID_ARG, "precond needs elses_mat_set_preconditioner first");
    }
    // M not SPD on the matrix (its M B interval has no positive lower end): the plain overlap solve
    const bool pre = want_pre && mat->mb_spd;
    ctx->last_products = 0;
    ctx->last_fallbacks = (want_pre && !pre) ? 1 : 0;
    if (traces_out) traces_out[0] = traces_out[1] = 0.0;
    if (n_cols == 0) return ELSES_OK;

    hipStream_t st = ctx->stream;
    // autotuned variant and slot count (global solves with both left at 0)
    {
        const int pk = o.use_mixed ? 1 : 0;
        if (!rp && o.variant == 0 && o.slots == 0 && mat->tuned_slots[pk] > 0) {
            o.variant = mat->tuned_variant[pk];
            o.slots = std::max(64, std::min(mat->tuned_slots[pk], ((n_cols + 63) / 64) * 64));
            if (o.slots > 128 && o.slots % 128 != 0) o.slots += 64;
        }
    }
    // ld: slots (columns advanced together); vw: width of a vector row
    const int ld = rp ? rp->n_tiles * rp->L : choose_slots(n_cols, M, o);
    const int vw = rp ? rp->L : ld;
    if (ld % 64 != 0) return set_err(ctx, ELSES_ERR_INVALID_ARG, "slot count must be a multiple of 64");
    PassArgs pa{};
    const char* verr = configure_pass(d, o.variant, vw, pa);
    if (verr) return set_err(ctx, ELSES_ERR_INVALID_ARG, verr);
    // region tiles: slabs of groups of one tile, chunks of slabs for the reductions
    std::vector<int> slab_group, slab_tile, chunk_s0, chunk_s1, tile_chunk_off;
    if (rp) {
        const char* rerr = region_slabs(rp, pa, slab_group, slab_tile, chunk_s0, chunk_s1, tile_chunk_off);
        if (rerr) return set_err(ctx, ELSES_ERR_INVALID_ARG, rerr);
    }
    const int n_groups = pa.n_slabs;
    const int* row_tile = rp ? rp->d_row_tile : nullptr;
    const bool mixed = o.use_mixed != 0;
    if (mixed && (pa.staged == 1 || pa.staged == 2))
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "the LDS-staged passes have no mixed-precision form");
    const double* valsA = (pa.staged == 9) ? d.grp.A : d.A;
    const double* valsB = (pa.staged == 9) ? d.grp.B : d.B;
    const float* valsA32 = (pa.staged == 9) ? d.grp.A32 : d.A32;
    const float* valsB32 = (pa.staged == 9) ? d.grp.B32 : d.B32;
    const int rmax = full ? M : h.pmax;
    // FP64: one Richardson solve to inner_tol.  Mixed: two FP32 rounds (the
    // solve, then the solve of the FP64 residual), each to sqrt(inner_tol).
    // the polynomial on B's interval, or with M on the interval of M B (x <- x + tau_k M (s - B x))
    const double ilo = pre ? mat->mb_lo : mat->b_lo, ihi = pre ? mat->mb_hi : mat->b_hi;
    const Rich rich = richardson_plan(ilo, ihi, mixed ? std::sqrt(o.inner_tol) : o.inner_tol);
    if (check_rich(ctx, rich, mixed ? std::sqrt(o.inner_tol) : o.inner_tol, ilo, ihi) != ELSES_OK)
        return ELSES_ERR_INVALID_ARG;

    // host-side pattern offsets
    std::vector<int64_t> row_off(n_cols + 1, 0);
    if (rp) {
        row_off = rp->pat_off;
    } else {
        std::vector<int> orb_atom(M);
        for (int I = 0; I < h.n_atoms; ++I)
            for (int q = h.atom_off[I]; q < h.atom_off[I + 1]; ++q) orb_atom[q] = I;
        for (int c = 0; c < n_cols; ++c)
            row_off[c + 1] = row_off[c] + (full ? (int64_t)M : (int64_t)h.atom_plen[orb_atom[cols[c]]]);
    }

    int n_notconv = 0;
    int* h_rem = nullptr;
    hipEvent_t ev = nullptr;
    try {
        HCHECK(hipSetDevice(ctx->device));
        DevPool pool;
        const size_t vsz = (size_t)M * vw;
        double* buf[5] = {};
        for (int i = 0; i < 5; ++i) {
            buf[i] = pool.get<double>(vsz);
            HCHECK(hipMemsetAsync(buf[i], 0, vsz * sizeof(double), st));
        }
        // the preconditioned steps' residual and M-product blocks
        double* Rpre = pre ? pool.get<double>(vsz) : nullptr;
        double* Qpre = pre ? pool.get<double>(vsz) : nullptr;
        float* buf32[6] = {};
        if (mixed)
            for (int i = 0; i < 6; ++i) {
                buf32[i] = pool.get<float>(vsz);
                HCHECK(hipMemsetAsync(buf32[i], 0, vsz * sizeof(float), st));
            }
        double* part0 = pool.get<double>((size_t)n_groups * vw);
        double* part1 = pool.get<double>((size_t)n_groups * vw);
        HCHECK(hipMemsetAsync(part0, 0, sizeof(double) * n_groups * vw, st));
        HCHECK(hipMemsetAsync(part1, 0, sizeof(double) * n_groups * vw, st));
        double* red_tmp = pool.get<double>(rp ? chunk_s0.size() * (size_t)vw : (size_t)((n_groups + 63) / 64) * ld);
        int *d_slab_group = nullptr, *d_slab_tile = nullptr, *d_chunk = nullptr, *d_tile_live = nullptr;
        if (rp) {
            d_slab_group = pool.get<int>(slab_group.size());
            d_slab_tile = pool.get<int>(slab_tile.size());
            d_chunk = pool.get<int>(2 * chunk_s0.size() + tile_chunk_off.size());
            HCHECK(hipMemcpyAsync(d_slab_group, slab_group.data(), sizeof(int) * slab_group.size(),
                                  hipMemcpyHostToDevice, st));
            HCHECK(hipMemcpyAsync(d_slab_tile, slab_tile.data(), sizeof(int) * slab_tile.size(), hipMemcpyHostToDevice,
                                  st));
            HCHECK(hipMemcpyAsync(d_chunk, chunk_s0.data(), sizeof(int) * chunk_s0.size(), hipMemcpyHostToDevice, st));
            HCHECK(hipMemcpyAsync(d_chunk + chunk_s0.size(), chunk_s1.data(), sizeof(int) * chunk_s1.size(),
                                  hipMemcpyHostToDevice, st));
            HCHECK(hipMemcpyAsync(d_chunk + 2 * chunk_s0.size(), tile_chunk_off.data(),
                                  sizeof(int) * tile_chunk_off.size(), hipMemcpyHostToDevice, st));
            pa.slab_group = d_slab_group;
            pa.slab_tile = d_slab_tile;
            // running columns per tile (region tiles have no refill)
            std::vector<int> live(rp->n_tiles, 0);
            for (int t = 0; t < rp->n_tiles; ++t)
                for (int c = 0; c < rp->L; ++c) live[t] += rp->slot_map[(size_t)t * rp->L + c] >= 0 ? 1 : 0;
            d_tile_live = pool.get<int>(live.size());
            HCHECK(hipMemcpyAsync(d_tile_live, live.data(), sizeof(int) * live.size(), hipMemcpyHostToDevice, st));
            pa.tile_live = d_tile_live;
        }
        double* vs = pool.get<double>(ld);
        double* ss = pool.get<double>(ld);
        double* alpha = pool.get<double>(ld);
        double* beta_prev = pool.get<double>(ld);
        double* inv_beta = pool.get<double>(ld);
        double* coefT = pool.get<double>(ld);
        int* slot_n = pool.get<int>(ld);
        int* slot_row = pool.get<int>(ld);
        int* slot_cidx = pool.get<int>(ld);
        double* eta = pool.get<double>((size_t)ld * K * 2);
        double* zeta = pool.get<double>((size_t)ld * K * 2);
        int* conv = pool.get<int>((size_t)ld * K);
        double* res = pool.get<double>((size_t)ld * K);
        double* xs = pool.get<double>((size_t)ld * K * rmax * 2);
        double* ps = pool.get<double>((size_t)ld * K * rmax * 2);
        int* d_cols = rp ? rp->d_col_row : pool.get<int>(n_cols);
        int64_t* d_row_off = rp ? rp->d_pat_off : pool.get<int64_t>(n_cols + 1);
        int* d_rows = rp ? rp->d_rows : (full ? nullptr : pool.get<int>((size_t)row_off[n_cols]));
        int64_t* d_vidx = rp ? rp->d_vidx : (density ? pool.get<int64_t>((size_t)row_off[n_cols]) : nullptr);
        double* d_z = pool.get<double>(2 * K);
        double* d_cw = density ? pool.get<double>(2 * K) : nullptr;
        int* counters = pool.get<int>(4);
        double* ctr = (density || col_traces_out) ? (col_traces_out ? col_traces_out : pool.get<double>(2 * (size_t)n_cols))
                                                  : nullptr;
        double* tr2 = pool.get<double>(2);
        HCHECK(hipMemsetAsync(conv, 0, sizeof(int) * ld * K, st));
        if (!rp) {
            HCHECK(hipMemcpyAsync(d_cols, cols, sizeof(int) * n_cols, hipMemcpyHostToDevice, st));
            HCHECK(hipMemcpyAsync(d_row_off, row_off.data(), sizeof(int64_t) * (n_cols + 1), hipMemcpyHostToDevice,
                                  st));
        }
        HCHECK(hipMemcpyAsync(d_z, shifts, sizeof(double) * 2 * K, hipMemcpyHostToDevice, st));
        if (density) HCHECK(hipMemcpyAsync(d_cw, cw, sizeof(double) * 2 * K, hipMemcpyHostToDevice, st));
        if (!full && !rp) launch_pattern_setup(d, n_cols, d_cols, d_row_off, d_rows, d_vidx, st);

        ShiftArgs sa{};
        sa.ld = ld;
        sa.vld = vw;
        sa.slot_map = rp ? rp->d_slot_map : nullptr;
        sa.tile_live = d_tile_live;
        sa.K = K;
        sa.M = M;
        sa.z = d_z;
        sa.cw = d_cw;
        sa.slot_n = slot_n;
        sa.slot_row = slot_row;
        sa.slot_cidx = slot_cidx;
        sa.beta_prev = beta_prev;
        sa.inv_beta = inv_beta;
        sa.coefT = coefT;
        sa.alpha = alpha;
        sa.vs = vs;
        sa.ss = ss;
        sa.eta = eta;
        sa.zeta = zeta;
        sa.conv = conv;
        sa.res = res;
        sa.xs = xs;
        sa.ps = ps;
        sa.rmax = rmax;
        sa.n_cols = n_cols;
        sa.cols = d_cols;
        sa.row_off = d_row_off;
        sa.rows = d_rows;
        sa.vidx = d_vidx;
        sa.Bv = gd.B;
        sa.Av = gd.A;
        sa.full = full ? 1 : 0;
        sa.tol = o.tol;
        sa.max_outer = o.max_outer;
        sa.queue = counters;
        sa.remaining = counters + 1;
        sa.n_notconv = counters + 2;
        sa.x_out = x_out;
        sa.iters_out = iters_out;
        sa.resid_out = o.audit ? nullptr : resid_out;
        sa.rho_out = rho_out;
        sa.ctr_out = ctr;
        launch_slot_init(sa, std::min(n_cols, ld), st);

        pa.inv_beta = inv_beta;
        pa.coefT = coefT;
        pa.alpha = alpha;
        pa.slot_n = slot_n;
        pa.slot_row = slot_row;
        pa.part0 = part0;
        pa.part1 = part1;
        pa.g0 = rich.g0;

        // column sums of the dot partials (masked: idle and starting slots get 0)
        auto reduce = [&](const double* part, double* out, bool masked) {
            const int* sn = masked ? slot_n : nullptr;
            const int* sr = masked ? slot_row : nullptr;
            if (rp)
                launch_col_reduce_tiles(part, vw, rp->n_tiles, (int)chunk_s0.size(), d_chunk,
                                        d_chunk + chunk_s0.size(), d_chunk + 2 * chunk_s0.size(), red_tmp, sn, sr,
                                        out, st);
            else
                launch_col_reduce(part, n_groups, ld, red_tmp, sn, sr, out, st);
        };
        HCHECK(hipHostMalloc((void**)&h_rem, sizeof(int) * 4, hipHostMallocDefault));
        HCHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        int64_t it = 0;
        // Sampled event timing of the overlap-solve passes.  A sample spans the back-to-back Richardson steps k = 2 .. d-2 of one
        // outer iteration (d - 3 launches of the same kernel), so the mean
        // launch time excludes the event overhead.
        struct EvPair {
            hipEvent_t a = nullptr, b = nullptr;
            bool busy = false;
            int n = 0;
        };
        std::vector<EvPair> prof(ctx->prof_stride > 0 ? 32 : 0);
        for (auto& p : prof) {
            HCHECK(hipEventCreate(&p.a));
            HCHECK(hipEventCreate(&p.b));
        }
        auto harvest = [&]() {
            for (auto& p : prof)
                if (p.busy && hipEventQuery(p.b) == hipSuccess) {
                    float ms = 0.f;
                    HCHECK(hipEventElapsedTime(&ms, p.a, p.b));
                    ctx->prof_ms += ms;
                    ctx->prof_launches += p.n;
                    p.busy = false;
                }
        };
        if (!prof.empty()) {
            const double w = mixed ? 4.0 : 8.0;  // bytes per value and per vector entry of the timed pass
            ctx->prof_bytes = (double)d.nnz * w + (double)d.nnzb * 4.0 + (double)d.n_atoms * 20.0 +
                              3.0 * (double)M * vw * w;
            ctx->prof_flops = 2.0 * (double)d.nnz * vw + 3.0 * (double)M * vw;
            ctx->prof_slots = ld;
        }
        EvPair* open_sample = nullptr;
        bool capturing = false;
        auto timed_pass = [&](PassKind kind, int k) {
            const int first = 2, last = rich.d - 2;
            if (k == first && last >= first && !prof.empty() && !capturing && it % ctx->prof_stride == 0)
                for (auto& p : prof)
                    if (!p.busy) {
                        open_sample = &p;
                        HCHECK(hipEventRecord(p.a, st));
                        break;
                    }
            launch_pass(kind, pa, st);
            if (k == last && open_sample) {
                HCHECK(hipEventRecord(open_sample->b, st));
                open_sample->busy = true;
                open_sample->n = last - first + 1;
                open_sample = nullptr;
            }
        };
        // Buffers: q_n, t_{n-1}, t_n and two free blocks.  Each outer step:
        // s' = A q_n - beta t_{n-1} overwrites t_{n-1}; the first overlap step
        // writes s = s' - alpha t_n to a free block; the Richardson iterates
        // ping-pong between the other free block and the s' block; then
        // q <- v, t_{n-1} <- t_n, t_n <- s.
        double* Vq = buf[0];
        double* Tp = buf[1];
        double* Tn = buf[2];
        double* F1 = buf[3];
        double* F2 = buf[4];
        float* S32 = buf32[0];
        float* Xa32 = buf32[1];
        float* Xb32 = buf32[2];
        float* R32 = buf32[3];
        float* Da32 = buf32[4];
        float* Db32 = buf32[5];
        const int poll = 8;
        const int64_t generations = (n_cols + ld - 1) / ld + 1;
        const int64_t cap = (int64_t)o.max_outer * generations + 64;
        bool pending = false;
        // one outer iteration: launches, then the rotation of the buffers
        auto iteration = [&]() {
                // w = A q_n, s' = w - beta t_{n-1} (in place of t_{n-1}), alpha_n
                pa.vals = valsA;
                pa.vals32 = valsA32;
                pa.Xg = Vq;
                pa.S = Tp;
                pa.Vq = Vq;
                launch_pass(mixed ? PASS_LANCZOS_A_MX : PASS_LANCZOS_A, pa, st);
                reduce(part0, alpha, true);
                // overlap solve v = p(B) s on s = s' - alpha t_n (Richardson steps
                // with the Chebyshev roots in Leja order)
                pa.vals = valsB;
                pa.vals32 = valsB32;
                pa.Tn = Tn;
                double* vout = nullptr;
                if (pre) {
                    // s = s' - alpha t_n into F1; x_1 = g0 M s, then
                    // x_{k+1} = x_k + tau_k M (s - B x_k), k = 1 .. d-1; v.s and s.s partials
                    const int64_t nv = (int64_t)M * vw;
                    launch_overlap_start(M, vw, Tp, Tn, alpha, inv_beta, row_tile, 0.0, F1, F2, nullptr, nullptr,
                                         st);
                    launch_spmm_generic(gd, mat->M_dev, ld, ld, F1, Qpre, st);
                    launch_axpby(nv, 0.0, nullptr, rich.g0, Qpre, F2, st);
                    double* xcur = F2;
                    double* xoth = Tp;
                    for (int k = 1; k < rich.d; ++k) {
                        launch_spmm_generic(gd, gd.B, ld, ld, xcur, Rpre, st);
                        launch_axpby(nv, 1.0, F1, -1.0, Rpre, Rpre, st);
                        launch_spmm_generic(gd, mat->M_dev, ld, ld, Rpre, Qpre, st);
                        launch_axpby(nv, 1.0, xcur, rich.tau[k - 1], Qpre, xoth, st);
                        std::swap(xcur, xoth);
                    }
                    launch_dots2_partial(M, ld, n_groups, xcur, F1, part0, part1, st);
                    vout = xcur;
                    F2 = xoth;
                } else if (!mixed) {
                    // s = s' - alpha t_n into F1, x_1 = g0 s into F2; then steps 1 .. d-1
                    launch_overlap_start(M, vw, Tp, Tn, alpha, inv_beta, row_tile, rich.g0, F1, F2, nullptr,
                                         nullptr, st);
                    double* xcur = F2;
                    double* xoth = Tp;
                    pa.S = F1;
                    for (int k = 1; k < rich.d; ++k) {
                        pa.Xg = xcur;
                        pa.Xio = xoth;
                        pa.tau = rich.tau[k - 1];
                        timed_pass(k == rich.d - 1 ? PASS_STEP_LAST : PASS_STEP, k);
                        std::swap(xcur, xoth);
                    }
                    vout = xcur;
                    F2 = xoth;
                } else {
                    // first FP32 solve: B x = s (s kept in FP64 and FP32)
                    launch_overlap_start(M, vw, Tp, Tn, alpha, inv_beta, row_tile, rich.g0, F1, nullptr, S32, Xa32,
                                         st);
                    float* xcur = Xa32;
                    float* xoth = Xb32;
                    pa.R32 = S32;
                    for (int k = 1; k < rich.d; ++k) {
                        pa.Xg32 = xcur;
                        pa.Xio32 = xoth;
                        pa.tau = rich.tau[k - 1];
                        timed_pass(PASS_STEP32, k);
                        std::swap(xcur, xoth);
                    }
                    // FP64 residual r = s - B x, first correction iterate
                    pa.S = F1;
                    pa.Xg32 = xcur;
                    pa.R32o = R32;
                    pa.Xio32 = Da32;
                    launch_pass(PASS_REFINE, pa, st);
                    // second FP32 solve, the correction: B d = r; the last step forms v = x + d
                    float* dcur = Da32;
                    float* doth = Db32;
                    pa.R32 = R32;
                    pa.Xr1 = xcur;
                    pa.Xio = F2;
                    for (int k = 1; k < rich.d; ++k) {
                        pa.Xg32 = dcur;
                        pa.Xio32 = doth;
                        pa.tau = rich.tau[k - 1];
                        launch_pass(k == rich.d - 1 ? PASS_STEP32_LAST : PASS_STEP32, pa, st);
                        std::swap(dcur, doth);
                    }
                    vout = F2;
                    F2 = Tp;
                }
                reduce(part0, vs, false);
                reduce(part1, ss, false);
                // multi-shift recurrences, convergence, slot refill
                sa.Vq = Vq;
                launch_shift_update(sa, st);
                HCHECK(hipGetLastError());
                // rotate: q <- v, t_{n-1} <- t_n, t_n <- s; the old q block is free
                double* oldV = Vq;
                Vq = vout;
                Tp = Tn;
                Tn = F1;
                F1 = oldV;
        };
        auto poll_done = [&]() -> bool {
            if (pending) {
                HCHECK(hipEventSynchronize(ev));
                harvest();
                if (h_rem[0] == 0) return true;
            }
            HCHECK(hipMemcpyAsync(h_rem, sa.remaining, sizeof(int), hipMemcpyDeviceToHost, st));
            HCHECK(hipEventRecord(ev, st));
            pending = true;
            return false;
        };
        if (!o.graph) {
            for (;;) {
                iteration();
                ++it;
                if (it % poll == 0 && poll_done()) break;
                if (it > cap) throw HipFail{hipErrorUnknown, "solver loop did not terminate"};
            }
        } else {
            // Capture G outer iterations (a whole number of periods of the
            // buffer rotation, at least `poll`) into one graph on a private
            // stream and replay it, polling between replays.
            const double* start[5] = {Vq, Tp, Tn, F1, F2};
            int period = 0;
            {
                double* p[5] = {Vq, Tp, Tn, F1, F2};
                for (int q = 1; q <= 12 && period == 0; ++q) {
                    // the rotation of `iteration` (FP64: v ends in F2 or the s' block by parity)
                    double* vout = mixed ? p[4] : ((rich.d - 1) % 2 == 0 ? p[4] : p[1]);
                    double* xoth = mixed ? p[1] : ((rich.d - 1) % 2 == 0 ? p[1] : p[4]);
                    double* nv[5] = {vout, p[2], p[3], p[0], xoth};
                    for (int r = 0; r < 5; ++r) p[r] = nv[r];
                    bool same = true;
                    for (int r = 0; r < 5; ++r) same = same && p[r] == start[r];
                    if (same) period = q;
                }
            }
            if (period == 0) throw HipFail{hipErrorUnknown, "buffer rotation has no short period"};
            const int G = period * ((poll + period - 1) / period);
            hipStream_t gs = nullptr;
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            hipEvent_t ready = nullptr;
            const hipStream_t st0 = st;
            auto cleanup = [&]() {
                if (exec) (void)hipGraphExecDestroy(exec);
                if (graph) (void)hipGraphDestroy(graph);
                if (ready) (void)hipEventDestroy(ready);
                if (gs) (void)hipStreamDestroy(gs);
                st = st0;
            };
            try {
                HCHECK(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking));
                HCHECK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
                HCHECK(hipEventRecord(ready, st0));
                HCHECK(hipStreamWaitEvent(gs, ready, 0));
                st = gs;  // every launch below (the lambdas capture st by reference)
                capturing = true;
                HCHECK(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
                for (int q = 0; q < G; ++q) iteration();
                HCHECK(hipStreamEndCapture(gs, &graph));
                capturing = false;
                for (int r = 0; r < 5; ++r)
                    if ((r == 0 ? Vq : r == 1 ? Tp : r == 2 ? Tn : r == 3 ? F1 : F2) != start[r])
                        throw HipFail{hipErrorUnknown, "graph capture did not return the buffers to their roles"};
                HCHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
                for (;;) {
                    HCHECK(hipGraphLaunch(exec, gs));
                    it += G;
                    if (poll_done()) break;
                    if (it > cap) throw HipFail{hipErrorUnknown, "solver loop did not terminate"};
                }
                HCHECK(hipEventRecord(ready, gs));
                HCHECK(hipStreamWaitEvent(st0, ready, 0));
                HCHECK(hipStreamSynchronize(gs));
            } catch (...) {
                if (capturing) {
                    hipGraph_t g2 = nullptr;
                    (void)hipStreamEndCapture(gs, &g2);
                    if (g2) (void)hipGraphDestroy(g2);
                    capturing = false;
                }
                cleanup();
                throw;
            }
            cleanup();
        }
        if (o.audit) launch_true_residual(d, mixed, n_cols, d_cols, K, d_z, x_out, resid_out, st);
        if (density) {
            launch_sum_pairs(ctr, n_cols, tr2, st);
            if (traces_out) HCHECK(hipMemcpyAsync(traces_out, tr2, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
        }
        HCHECK(hipMemcpyAsync(h_rem, counters, sizeof(int) * 3, hipMemcpyDeviceToHost, st));
        HCHECK(hipStreamSynchronize(st));
        HCHECK(hipGetLastError());
        harvest();
        for (auto& p : prof) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
        ctx->total_passes += it * (mixed ? 2 * rich.d : rich.d);
        n_notconv = h_rem[2];
        (void)hipEventDestroy(ev);
        (void)hipHostFree(h_rem);
    } catch (const HipFail& f) {
        if (ev) (void)hipEventDestroy(ev);
        if (h_rem) (void)hipHostFree(h_rem);
        const elses_status s = (f.e == hipErrorOutOfMemory) ? ELSES_ERR_OOM : ELSES_ERR_HIP;
        return set_err(ctx, s, std::string(f.what) + ": " + hipGetErrorString(f.e));
    }
    if (n_notconv > 0) {
        return set_err(ctx, ELSES_WARN_NOT_CONVERGED,
                       std::to_string(n_notconv) + " column(s) reached max_outer before every shift converged");
    }
    return ELSES_OK;
}

// Device work buffers of one call: from a DevPool (allocated and freed per
// call), or carved from a fixed arena (the allocation-free entry point), in
// 256-byte aligned pieces.
struct Scratch {
    DevPool* pool = nullptr;
    char* base = nullptr;
    size_t cap = 0, used = 0;
    template <typename T>
    T* get(size_t n) {
        if (pool) return pool->get<T>(n);
        const size_t bytes = ((std::max<size_t>(n, 1) * sizeof(T)) + 255) & ~(size_t)255;
        if (used + bytes > cap) throw HipFail{hipErrorOutOfMemory, "no-allocation scratch exhausted"};
        T* p = reinterpret_cast<T*>(base + used);
        used += bytes;
        return p;
    }
};

size_t round256(size_t b) { return (std::max<size_t>(b, 1) + 255) & ~(size_t)255; }

// Region solves in the compact layout: argument checks, scratch, one
// persistent launch per column-width group (region.hip), then the trace sum.
// With an arena (the allocation-free entry point) every work buffer comes
// from it, the groups run one after another on the context stream with as
// many workgroups as the arena holds, and no stream, event or allocation is
// created.
constexpr int kRegionsPerCu = 1;  // resident workgroups per CU of a compact launch

// Overlap interval of region r of a compact set: the extreme Ritz values of
// its B widened like B's own interval (2 % of the width and 1e-3 relative on
// each side) and kept inside B's interval.
void region_interval(const elses_regions_s* rp, int r, double& lo, double& hi) {
    const double tl = rp->cp.ritz_lo[r], th = rp->cp.ritz_hi[r], w = th - tl;
    lo = std::max(rp->gm->b_lo, tl - 0.02 * w - 1e-3 * std::fabs(tl));
    hi = std::min(rp->gm->b_hi, th + 0.02 * w + 1e-3 * std::fabs(th));
}

elses_status compact_solve(elses_ctx ctx, const elses_regions_s* rp, int K, const double* shifts, const double* cw,
                           const elses_opts* opts_in, double* x_out, int32_t* iters_out, double* resid_out,
                           double* rho_out, double* traces_out, double* col_traces_out, char* arena = nullptr,
                           size_t arena_bytes = 0) {
    elses_opts o;
    elses_opts_default(&o);
    if (opts_in) o = *opts_in;
    const elses_mat mat = rp->gm;
    const auto& C = rp->cp;
    const bool density = (cw != nullptr);
    const int n_cols = rp->n_cols;
    if (K < 1 || K > 256) return set_err(ctx, ELSES_ERR_INVALID_ARG, "n_shifts must be in [1, 256]");
    if (!shifts) return set_err(ctx, ELSES_ERR_INVALID_ARG, "shifts is null");
    for (int k = 0; k < K; ++k) {
        if (!std::isfinite(shifts[2 * k]) || !std::isfinite(shifts[2 * k + 1]) || !(shifts[2 * k + 1] > 0.0))
            return set_err(ctx, ELSES_ERR_INVALID_ARG, "every shift needs a finite value with Im z > 0");
        if (density && (!std::isfinite(cw[2 * k]) || !std::isfinite(cw[2 * k + 1])))
            return set_err(ctx, ELSES_ERR_INVALID_ARG, "non-finite density weight");
    }
    if (!(o.tol > 0.0) || !std::isfinite(o.tol)) return set_err(ctx, ELSES_ERR_INVALID_ARG, "tol must be > 0");
    if (o.max_outer < 1) return set_err(ctx, ELSES_ERR_INVALID_ARG, "max_outer must be >= 1");
    if (!(o.inner_tol > 0.0 && o.inner_tol < 1.0))
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "inner_tol must be in (0, 1)");
    if (o.out_mode != ELSES_OUT_PATTERN && o.out_mode != ELSES_OUT_FULL)
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "out_mode must be PATTERN or FULL");
    if (o.use_mixed && !C.has32)
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "use_mixed needs a matrix created with ELSES_MIXED");
    const bool full = (o.out_mode == ELSES_OUT_FULL);
    if (full && density)
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "density matrix output uses the pattern mode");
    if (o.audit && (!full || !resid_out))
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "audit needs ELSES_OUT_FULL and resid_out");
    if (o.audit_every < 0) return set_err(ctx, ELSES_ERR_INVALID_ARG, "audit_every must be >= 0");
    const bool precond = o.precond != 0;
    if (precond && !C.hasM)
        return set_err(ctx, ELSES_ERR_INVALID_ARG,
                       "precond needs a region set created after elses_mat_set_preconditioner");
    if (precond && o.inner_max < 1) return set_err(ctx, ELSES_ERR_INVALID_ARG, "inner_max must be >= 1");
    if (o.audit_every > 0 && (full || !resid_out))
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "audit_every needs the pattern mode and resid_out");
    if (traces_out) traces_out[0] = traces_out[1] = 0.0;
    const bool mixed = o.use_mixed != 0;
    const Rich rich = richardson_plan(mat->b_lo, mat->b_hi, mixed ? std::sqrt(o.inner_tol) : o.inner_tol);
    if (check_rich(ctx, rich, mixed ? std::sqrt(o.inner_tol) : o.inner_tol, mat->b_lo, mat->b_hi) != ELSES_OK)
        return ELSES_ERR_INVALID_ARG;
    // the Richardson plan of each region on its own overlap interval: the
    // extreme Ritz values of its B, widened like B's own interval and kept
    // inside it (a region's B is a principal submatrix of B, so its spectrum
    // lies inside B's); never a higher degree than B's plan
    const int n_reg = rp->n_regions;
    const double round_tol = mixed ? std::sqrt(o.inner_tol) : o.inner_tol;
    const int tau_stride = std::max(1, rich.d - 1);
    std::vector<int> h_rdeg(n_reg);
    std::vector<double> h_rg0(n_reg), h_rtau((size_t)n_reg * tau_stride, 0.0);
    for (int r = 0; r < n_reg; ++r) {
        double lo = 0.0, hi = 0.0;
        region_interval(rp, r, lo, hi);
        Rich pr = (lo > 0.0 && hi > lo) ? richardson_plan(lo, hi, round_tol) : rich;
        if (pr.d > rich.d || pr.reached > round_tol * (1.0 + 1e-12)) pr = rich;
        h_rdeg[r] = pr.d;
        h_rg0[r] = pr.g0;
        std::copy(pr.tau.begin(), pr.tau.end(), h_rtau.begin() + (size_t)r * tau_stride);
    }
    // one launch per vector-width group: LDS of its largest iterate, resident workgroups
    // (two iterate buffers when that keeps as many workgroups resident as one)
    size_t glds[3] = {0, 0, 0};
    int gwg[3] = {0, 0, 0}, ghalf[3] = {0, 0, 0}, gsym[3] = {0, 0, 0};
    for (int g = 0; g < 3; ++g) {
        const int cnt = C.goff[g + 1] - C.goff[g];
        if (cnt == 0) continue;
        glds[g] = (size_t)C.gmaxP[g] * C.gcw[g] * (mixed ? 4 : 8);
        const int occ = compact_occupancy(!mixed, C.gcw[g], precond, glds[g]);
        if (occ < 1)
            return set_err(ctx, ELSES_ERR_INVALID_ARG,
                           "the largest region's overlap iterate does not fit in LDS; use tile_width 64 or 128");
        if (compact_occupancy(!mixed, C.gcw[g], precond, 2 * glds[g]) >= occ) {
            ghalf[g] = C.gmaxP[g] * C.gcw[g];
            glds[g] *= 2;
            // FP32 Richardson steps on the half layout of B: a 32-bit fixed-point
            // transpose accumulator per position and column after the two iterate buffers.
            // Column widths 1 and 2 only: each stored pair costs one LDS atomic per
            // column, and at 4 columns the atomics outweigh the halved stream (a
            // 4-column region of the 10^6-atom benchmark ran 10.7 s against 7.0 s)
            const size_t ys = (size_t)C.gmaxP[g] * C.gcw[g] * 4;
            if (mixed && !precond && C.d_hidx && C.gcw[g] <= 2 &&
                compact_occupancy(false, C.gcw[g], false, glds[g] + ys) >= std::min(occ, kRegionsPerCu)) {
                gsym[g] = 1;
                glds[g] += ys;
            }
        }
        // at most one workgroup (one region) per CU: on the 10^6-atom benchmark the
        // solve ran 9.9 s per step with 256 resident regions against 11.0 s with 512,
        // with the same kernel; half as many resident region matrices stay in the
        // last-level cache between their products
        gwg[g] = std::max(1, std::min(cnt, std::min(occ, kRegionsPerCu) * ctx->n_cu));
    }
    // carried rows per column: the pattern, or every position of the region (full output, audits)
    std::vector<int> carry_full(n_cols, 0);
    std::vector<int64_t> carry_off(n_cols + 1, 0), full_off(n_cols + 1, 0);
    for (int c = 0; c < n_cols; ++c) {
        const RegionDesc& D = C.reg[C.col_region[c]];
        carry_full[c] = (full || (o.audit_every > 0 && c % o.audit_every == 0)) ? 1 : 0;
        const int64_t len = carry_full[c] ? (int64_t)D.nslice * 64 : rp->pat_off[c + 1] - rp->pat_off[c];
        carry_off[c + 1] = carry_off[c] + len * K;
        full_off[c + 1] = full_off[c] + D.m;
    }
    // per-workgroup scratch of each group: seven [P][cw] FP64 blocks (twelve with the
    // preconditioned solve's own vectors)
    const size_t nblk = precond ? 12 : 7;
    const bool noalloc = arena != nullptr;
    if (noalloc) {
        // fixed part of the arena, in the order and rounding of the gets below
        size_t fixed = round256(sizeof(int64_t) * (n_cols + 1)) * 2 + round256(sizeof(int) * n_cols) +
                       round256(sizeof(double) * 2 * K) * (density ? 2 : 1) +
                       round256(sizeof(int) * n_reg) + round256(sizeof(double) * n_reg) +
                       round256(sizeof(double) * n_reg * tau_stride) +
                       round256(sizeof(double) * n_cols * K * 2) * 2 + round256(sizeof(double) * n_cols * K) +
                       round256(sizeof(double) * n_cols * K * 4) + round256(sizeof(int) * n_cols * K) +
                       round256(sizeof(double) * carry_off[n_cols] * 2) * 2 + round256(sizeof(int) * 8) +
                       (iters_out ? 0 : round256(sizeof(int32_t) * n_cols)) +
                       ((density && !col_traces_out && traces_out) ? round256(sizeof(double) * 2 * n_cols) : 0) +
                       ((density && traces_out) ? round256(sizeof(double) * 2) : 0);
        // the groups run one after another and share the per-workgroup blocks
        size_t need_one = 0;
        for (int g = 0; g < 3; ++g)
            if (gwg[g] > 0) need_one = std::max(need_one, nblk * C.gmaxP[g] * C.gcw[g] * sizeof(double));
        if (fixed + round256(need_one) > arena_bytes)
            return set_err(ctx, ELSES_ERR_INVALID_ARG,
                           "the solve needs " + std::to_string(fixed + need_one) +
                               " bytes of scratch; the allocation-free entry point holds " +
                               std::to_string(arena_bytes) + " (use fewer columns or shifts per call)");
        const size_t room = arena_bytes - fixed - 256;
        for (int g = 0; g < 3; ++g) {
            if (gwg[g] == 0) continue;
            const size_t per = nblk * C.gmaxP[g] * C.gcw[g] * sizeof(double);
            gwg[g] = (int)std::max<size_t>(1, std::min<size_t>((size_t)gwg[g], room / per));
        }
    }
    size_t gvec[3] = {0, 0, 0};
    for (int g = 0; g < 3; ++g) gvec[g] = nblk * C.gmaxP[g] * C.gcw[g] * gwg[g];
    int n_notconv = 0;
    try {
        HCHECK(hipSetDevice(ctx->device));
        hipStream_t st = ctx->stream;
        DevPool dpool;
        Scratch pool;
        if (noalloc) {
            pool.base = arena;
            pool.cap = arena_bytes;
        } else {
            pool.pool = &dpool;
        }
        CompactArgs a{};
        a.reg = C.d_reg;
        a.order = C.d_order;
        a.n_regions = rp->n_regions;
        a.slice_len = C.d_slice_len;
        a.slice_ent = C.d_slice_ent;
        a.idx = C.d_idx;
        a.A64 = C.d_A64;
        a.B64 = C.d_B64;
        a.A32 = C.d_A32;
        a.B32 = C.d_B32;
        a.M64 = C.d_M64;
        a.M32 = C.d_M32;
        a.inner_tol = o.inner_tol;
        a.inner_max = o.inner_max;
        a.pos_row = C.d_pos_row;
        a.hslice_len = C.d_hslice_len;
        a.hslice_ent = C.d_hslice_ent;
        a.hidx = C.d_hidx;
        a.hval = C.d_hval;
        a.hdiag = C.d_hdiag;
        a.col_pos = C.d_col_pos;
        a.pat_off = C.d_pat_off;
        a.pat_pos = C.d_pat_pos;
        a.pat_B = C.d_pat_B;
        a.pat_A = C.d_pat_A;
        int64_t* d_carry_off = pool.get<int64_t>(n_cols + 1);
        int* d_carry_full = pool.get<int>(n_cols);
        int64_t* d_full_off = pool.get<int64_t>(n_cols + 1);
        HCHECK(hipMemcpyAsync(d_carry_off, carry_off.data(), sizeof(int64_t) * (n_cols + 1), hipMemcpyHostToDevice,
                              st));
        HCHECK(hipMemcpyAsync(d_carry_full, carry_full.data(), sizeof(int) * n_cols, hipMemcpyHostToDevice, st));
        HCHECK(hipMemcpyAsync(d_full_off, full_off.data(), sizeof(int64_t) * (n_cols + 1), hipMemcpyHostToDevice,
                              st));
        a.carry_off = d_carry_off;
        a.carry_full = d_carry_full;
        a.full_off = d_full_off;
        a.full_out = full ? 1 : 0;
        a.audit = (o.audit || o.audit_every > 0) ? 1 : 0;
        a.K = K;
        double* d_z = pool.get<double>(2 * K);
        HCHECK(hipMemcpyAsync(d_z, shifts, sizeof(double) * 2 * K, hipMemcpyHostToDevice, st));
        a.z = d_z;
        double* d_cw = nullptr;
        if (density) {
            d_cw = pool.get<double>(2 * K);
            HCHECK(hipMemcpyAsync(d_cw, cw, sizeof(double) * 2 * K, hipMemcpyHostToDevice, st));
        }
        a.cw = d_cw;
        a.tol = o.tol;
        a.max_outer = o.max_outer;
        int* d_rdeg = pool.get<int>(n_reg);
        double* d_rg0 = pool.get<double>(n_reg);
        double* d_rtau = pool.get<double>((size_t)n_reg * tau_stride);
        HCHECK(hipMemcpyAsync(d_rdeg, h_rdeg.data(), sizeof(int) * n_reg, hipMemcpyHostToDevice, st));
        HCHECK(hipMemcpyAsync(d_rg0, h_rg0.data(), sizeof(double) * n_reg, hipMemcpyHostToDevice, st));
        HCHECK(hipMemcpyAsync(d_rtau, h_rtau.data(), sizeof(double) * h_rtau.size(), hipMemcpyHostToDevice, st));
        a.rdeg = d_rdeg;
        a.rg0 = d_rg0;
        a.rtau = d_rtau;
        a.tau_stride = tau_stride;
        a.eta = pool.get<double>((size_t)n_cols * K * 2);
        a.zeta = pool.get<double>((size_t)n_cols * K * 2);
        a.res = pool.get<double>((size_t)n_cols * K);
        a.fac = pool.get<double>((size_t)n_cols * K * 4);
        a.conv = pool.get<int>((size_t)n_cols * K);
        launch_zero_ints(a.conv, (size_t)n_cols * K, st);
        a.xs = pool.get<double>((size_t)carry_off[n_cols] * 2);
        a.ps = pool.get<double>((size_t)carry_off[n_cols] * 2);
        int* counters = pool.get<int>(8);  // three queues, not-converged, fallbacks, pad, product count
        launch_zero_ints(counters, 8, st);
        a.n_notconv = counters + 3;
        a.n_fallback = counters + 4;
        a.products = reinterpret_cast<unsigned long long*>(counters + 6);
        a.x_out = x_out;
        int32_t* iters = iters_out ? iters_out : pool.get<int32_t>(n_cols);
        a.iters_out = iters;
        a.resid_out = resid_out;
        a.rho_out = rho_out;
        double* ctr = col_traces_out;
        if (density && !ctr && traces_out) ctr = pool.get<double>(2 * (size_t)n_cols);
        a.ctr_out = density ? ctr : nullptr;
        double* tr2 = (density && traces_out && ctr) ? pool.get<double>(2) : nullptr;
        // per-workgroup blocks last: in the arena the groups share one buffer
        double* vec_g[3] = {nullptr, nullptr, nullptr};
        if (noalloc) {
            size_t most = 0;
            for (int g = 0; g < 3; ++g) most = std::max(most, gvec[g]);
            double* shared = most ? pool.get<double>(most) : nullptr;
            for (int g = 0; g < 3; ++g) vec_g[g] = gvec[g] ? shared : nullptr;
        } else {
            for (int g = 0; g < 3; ++g)
                if (gvec[g] > 0) vec_g[g] = pool.get<double>(gvec[g]);
        }
        // One launch per group, on streams of their own (default priority) so
        // that a group's last regions overlap the next group's work: the
        // widest regions (longest per region) start first.  HIP events around
        // each launch when profiling is enabled.
        hipEvent_t ev[3][2] = {};
        const bool timed = ctx->prof_stride > 0 && !noalloc;
        unsigned long long* clk[3] = {nullptr, nullptr, nullptr};  // per-workgroup start / end stamps
        hipStream_t gst[3] = {st, st, st};
        hipStream_t own[3] = {nullptr, nullptr, nullptr};  // streams created here
        hipEvent_t ready = nullptr, gdone[3] = {};
        struct StreamGuard {
            hipStream_t* s;
            hipEvent_t* e;
            hipEvent_t* r;
            ~StreamGuard() {
                for (int g = 0; g < 3; ++g)
                    if (s[g]) (void)hipStreamDestroy(s[g]);
                for (int g = 0; g < 3; ++g)
                    if (e[g]) (void)hipEventDestroy(e[g]);
                if (*r) (void)hipEventDestroy(*r);
            }
        } guard{own, gdone, &ready};
        if (!noalloc) {
            HCHECK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
            HCHECK(hipEventRecord(ready, st));
        }
        for (int g = 0; g < 3; ++g) {
            const int cnt = C.goff[g + 1] - C.goff[g];
            if (cnt == 0) continue;
            if (!noalloc && g > 0) {
                HCHECK(hipStreamCreateWithFlags(&own[g], hipStreamNonBlocking));
                gst[g] = own[g];
                HCHECK(hipStreamWaitEvent(gst[g], ready, 0));
            }
            a.order = C.d_order + C.goff[g];
            a.n_regions = cnt;
            a.lds_half = ghalf[g];
            a.half = gsym[g];
            a.queue = counters + g;
            a.vec = vec_g[g];
            a.vec_stride = nblk * C.gmaxP[g] * C.gcw[g];
            a.wg_clock = nullptr;
            if (timed) {
                clk[g] = pool.get<unsigned long long>(2 * (size_t)gwg[g]);
                a.wg_clock = clk[g];
                HCHECK(hipEventCreate(&ev[g][0]));
                HCHECK(hipEventCreate(&ev[g][1]));
                HCHECK(hipEventRecord(ev[g][0], gst[g]));
            }
            launch_compact(a, !mixed, C.gcw[g], precond, gwg[g], glds[g], gst[g]);
            HCHECK(hipGetLastError());
            if (timed) HCHECK(hipEventRecord(ev[g][1], gst[g]));
            if (g > 0 && !noalloc) {
                HCHECK(hipEventCreateWithFlags(&gdone[g], hipEventDisableTiming));
                HCHECK(hipEventRecord(gdone[g], gst[g]));
                HCHECK(hipStreamWaitEvent(st, gdone[g], 0));
            }
        }
        if (tr2) {
            launch_sum_pairs(ctr, n_cols, tr2, st);
            HCHECK(hipMemcpyAsync(traces_out, tr2, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
        }
        int h_cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        HCHECK(hipMemcpyAsync(h_cnt, counters, sizeof(int) * 8, hipMemcpyDeviceToHost, st));
        HCHECK(hipStreamSynchronize(st));
        n_notconv = h_cnt[3];
        unsigned long long prods = 0;
        memcpy(&prods, h_cnt + 6, sizeof(prods));
        ctx->last_products = (int64_t)prods;
        ctx->last_fallbacks = h_cnt[4];
        // algorithmic bytes of the launch: per outer step of a region, its
        // sparse products (index + value per nonzero), the carried x and p
        // (read and written), and the Lanczos vectors in scratch
        std::vector<int32_t> it_h(n_cols);
        HCHECK(hipMemcpy(it_h.data(), iters, sizeof(int32_t) * n_cols, hipMemcpyDeviceToHost));
        const double vb = mixed ? 4.0 : 8.0;
        double gbytes[3] = {0, 0, 0}, gflops[3] = {0, 0, 0};
        int64_t outer = 0;
        for (int r = 0; r < rp->n_regions; ++r) {
            const RegionDesc& D = C.reg[r];
            const int g = D.cw == 4 ? 0 : (D.cw == 2 ? 1 : 2);
            int n_it = 0;
            double carried = 0.0;
            for (int c = D.col0; c < D.col0 + D.ncol; ++c) {
                n_it = std::max(n_it, (int)it_h[c]);
                carried += (double)(carry_off[c + 1] - carry_off[c]);
            }
            const double nnz = (double)C.region_nnz[r];
            const double products = mixed ? (2.0 * (h_rdeg[r] - 1) + 1.0) : (double)(h_rdeg[r] - 1);
            // Richardson products (2 (d - 1) mixed, d - 1 FP64), the rest (refinement, A) on the full layout;
            // a half-layout product reads each stored pair once (index + value) and the diagonal
            const double rich = mixed ? 2.0 * (h_rdeg[r] - 1) : (double)(h_rdeg[r] - 1);
            const double full_b = nnz * (2.0 + vb);
            const double rich_b = gsym[g] ? (double)C.region_hnnz[r] * (2.0 + vb) + 4.0 * D.m : full_b;
            const double per_it = rich_b * rich + full_b * (products + 1.0 - rich) + 64.0 * carried +
                                  18.0 * 8.0 * (double)D.m * D.cw;
            gbytes[g] += (n_it + 1) * per_it;
            gflops[g] += (n_it + 1) * (2.0 * nnz * D.cw * (products + 1.0));
            outer += n_it;
        }
        if (timed) {
            // The group launches overlap on their streams: one solve counts as one
            // launch spanning the first launch's start to the last one's end, with
            // the algorithmic bytes of all groups; slots = the width of the group
            // that moved most bytes.
            int gfirst = -1, glast = -1, gmost = -1;
            float span = 0.f;
            for (int g = 0; g < 3; ++g) {
                if (!ev[g][0]) continue;
                if (gfirst < 0) gfirst = g;
                if (gmost < 0 || gbytes[g] > gbytes[gmost]) gmost = g;
            }
            for (int g = 0; g < 3; ++g) {
                if (!ev[g][0]) continue;
                float ms = 0.f;
                HCHECK(hipEventElapsedTime(&ms, ev[gfirst][0], ev[g][1]));
                if (ms > span) {
                    span = ms;
                    glast = g;
                }
            }
            if (gfirst >= 0 && glast >= 0) {
                ctx->prof_ms += span;
                ctx->prof_launches += 1;
                ctx->prof_bytes_acc += gbytes[0] + gbytes[1] + gbytes[2];
                ctx->prof_flops_acc += gflops[0] + gflops[1] + gflops[2];
                ctx->prof_bytes = ctx->prof_bytes_acc / (double)ctx->prof_launches;
                ctx->prof_flops = ctx->prof_flops_acc / (double)ctx->prof_launches;
                ctx->prof_slots = C.gcw[gmost];
                // idle share of the group that moves most bytes: 1 - (summed
                // lifetimes of its workgroups) / (its workgroups x span of the
                // solve).  The small groups' few workgroups end early by design
                // (one region each) and are not counted.
                uint64_t t0 = ~0ull, t1 = 0;
                double busy = 0.0;
                std::vector<unsigned long long> hc;
                for (int g = 0; g < 3; ++g) {
                    if (!clk[g]) continue;
                    hc.resize(2 * (size_t)gwg[g]);
                    HCHECK(hipMemcpy(hc.data(), clk[g], sizeof(unsigned long long) * hc.size(),
                                     hipMemcpyDeviceToHost));
                    for (int w = 0; w < gwg[g]; ++w) {
                        t0 = std::min<uint64_t>(t0, hc[2 * w]);
                        t1 = std::max<uint64_t>(t1, hc[2 * w + 1]);
                        if (g == gmost) busy += (double)(hc[2 * w + 1] - hc[2 * w]);
                    }
                }
                if (t1 > t0 && clk[gmost]) {
                    ctx->prof_idle_acc += 1.0 - busy / (gwg[gmost] * (double)(t1 - t0));
                    ctx->prof_idle_n += 1;
                }
            }
            for (auto& e : ev)
                for (hipEvent_t x : e)
                    if (x) (void)hipEventDestroy(x);
        }
        ctx->total_passes += outer;
    } catch (const HipFail& f) {
        const elses_status s = (f.e == hipErrorOutOfMemory) ? ELSES_ERR_OOM : ELSES_ERR_HIP;
        return set_err(ctx, s, std::string(f.what) + ": " + hipGetErrorString(f.e));
    }
    if (n_notconv > 0)
        return set_err(ctx, ELSES_WARN_NOT_CONVERGED,
                       std::to_string(n_notconv) + " column(s) reached max_outer before every shift converged");
    return ELSES_OK;
}

}  // namespace

extern "C" {

elses_status elses_shifted_solve(elses_ctx ctx, elses_mat mat, int32_t n_cols, const int32_t* cols,
                                 int32_t n_shifts, const double* shifts, const elses_opts* opts, double* x_out,
                                 int32_t* iters_out, double* resid_out) {
    return solve_core(ctx, mat, n_cols, cols, n_shifts, shifts, nullptr, opts, x_out, iters_out, resid_out, nullptr,
                      nullptr, nullptr);
}

elses_status elses_density_matrix(elses_ctx ctx, elses_mat mat, int32_t n_cols, const int32_t* cols,
                                  int32_t n_shifts, const double* shifts, const double* c, const elses_opts* opts,
                                  double* rho_out, double* traces_out, double* col_traces_out, double* x_out,
                                  int32_t* iters_out, double* resid_out) {
    if (!c) return set_err(ctx, ELSES_ERR_INVALID_ARG, "weights c are null");
    return solve_core(ctx, mat, n_cols, cols, n_shifts, shifts, c, opts, x_out, iters_out, resid_out, rho_out,
                      traces_out, col_traces_out);
}

elses_status elses_ctx_set_profiling(elses_ctx ctx, int32_t stride) {
    if (!ctx || stride < 0) return ELSES_ERR_INVALID_ARG;
    ctx->prof_stride = stride;
    ctx->prof_launches = 0;
    ctx->prof_ms = 0.0;
    ctx->prof_bytes_acc = 0.0;
    ctx->prof_flops_acc = 0.0;
    ctx->prof_idle_acc = 0.0;
    ctx->prof_idle_n = 0;
    ctx->total_passes = 0;
    return ELSES_OK;
}

elses_status elses_ctx_pass_stats(elses_ctx ctx, int64_t* launches, double* avg_us, double* bytes, double* flops,
                                  int64_t* total_passes, int32_t* slots) {
    if (!ctx) return ELSES_ERR_INVALID_ARG;
    if (launches) *launches = ctx->prof_launches;
    if (avg_us) *avg_us = ctx->prof_launches ? 1000.0 * ctx->prof_ms / ctx->prof_launches : 0.0;
    if (bytes) *bytes = ctx->prof_bytes;
    if (flops) *flops = ctx->prof_flops;
    if (total_passes) *total_passes = ctx->total_passes;
    if (slots) *slots = ctx->prof_slots;
    return ELSES_OK;
}

elses_status elses_ctx_region_idle(elses_ctx ctx, double* idle_share, int64_t* solves) {
    if (!ctx) return ELSES_ERR_INVALID_ARG;
    if (idle_share) *idle_share = ctx->prof_idle_n ? ctx->prof_idle_acc / (double)ctx->prof_idle_n : 0.0;
    if (solves) *solves = ctx->prof_idle_n;
    return ELSES_OK;
}

elses_status elses_time_pass(elses_ctx ctx, elses_mat mat, int32_t kind, int32_t variant, int32_t slots,
                             int32_t reps, double* avg_us) {
    if (!ctx || !mat || !avg_us) return ELSES_ERR_INVALID_ARG;
    if (kind < 0 || kind >= kPassKinds || reps < 1) return set_err(ctx, ELSES_ERR_INVALID_ARG, "bad kind or reps");
    const bool k32 = (kind >= PASS_LANCZOS_A_MX && kind <= PASS_PLAIN32) || kind == PASS_STEP32_FIRST;
    if (k32 && mat->precision != ELSES_MIXED)
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "mixed-precision passes need a matrix created with ELSES_MIXED");
    const DevMatrix& d = mat->d;
    PassArgs pa{};
    const char* verr = configure_pass(d, variant, slots, pa);
    if (verr) return set_err(ctx, ELSES_ERR_INVALID_ARG, verr);
    if (k32 && (pa.staged == 1 || pa.staged == 2))
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "the LDS-staged passes have no mixed-precision form");
    hipStream_t st = ctx->stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    try {
        DevPool pool;
        const size_t vsz = (size_t)d.M * slots;
        double* X = pool.get<double>(vsz);
        double* Y = pool.get<double>(vsz);
        double* S = pool.get<double>(vsz);
        double* V = pool.get<double>(vsz);
        double* T = pool.get<double>(vsz);
        for (double* p : {X, Y, S, V, T}) HCHECK(hipMemsetAsync(p, 0, vsz * sizeof(double), st));
        float* F[4];
        for (int i = 0; i < 4; ++i) {
            F[i] = k32 ? pool.get<float>(vsz) : nullptr;
            if (F[i]) HCHECK(hipMemsetAsync(F[i], 0, vsz * sizeof(float), st));
        }
        double* part0 = pool.get<double>((size_t)pa.n_slabs * slots);
        double* part1 = pool.get<double>((size_t)pa.n_slabs * slots);
        double* sc = pool.get<double>((size_t)3 * slots);
        int* si = pool.get<int>((size_t)2 * slots);
        HCHECK(hipMemsetAsync(sc, 0, sizeof(double) * 3 * slots, st));
        HCHECK(hipMemsetAsync(si, 0, sizeof(int) * 2 * slots, st));
        pa.vals = (pa.staged == 9) ? d.grp.B : d.B;
        pa.vals32 = (pa.staged == 9) ? d.grp.B32 : d.B32;
        pa.Xg = X;
        pa.Xio = Y;
        pa.S = S;
        pa.Vq = V;
        pa.Tn = T;
        pa.Sout = V;
        pa.Xg32 = F[0];
        pa.Xio32 = F[1];
        pa.R32 = F[2];
        pa.R32o = F[2];
        pa.Xr1 = F[3];
        pa.inv_beta = sc;
        pa.coefT = sc + slots;
        pa.alpha = sc + 2 * slots;
        pa.slot_n = si;
        pa.slot_row = si + slots;
        pa.part0 = part0;
        pa.part1 = part1;
        pa.tau = 0.5;
        pa.g0 = 0.5;
        const PassKind pk = static_cast<PassKind>(kind);
        launch_pass(pk, pa, st);  // warm-up
        HCHECK(hipEventCreate(&e0));
        HCHECK(hipEventCreate(&e1));
        HCHECK(hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r) launch_pass(pk, pa, st);
        HCHECK(hipEventRecord(e1, st));
        HCHECK(hipEventSynchronize(e1));
        HCHECK(hipGetLastError());
        float ms = 0.f;
        HCHECK(hipEventElapsedTime(&ms, e0, e1));
        *avg_us = 1000.0 * ms / reps;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    } catch (const HipFail& f) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return set_err(ctx, ELSES_ERR_HIP, std::string(f.what) + ": " + hipGetErrorString(f.e));
    }
    return ELSES_OK;
}

elses_status elses_regions_create(elses_ctx ctx, elses_mat mat, int32_t n_regions, const int32_t* centres,
                                  const double* radii, int32_t tile_width, elses_regions* out) {
    if (!ctx || !mat || !out) return ELSES_ERR_INVALID_ARG;
    *out = nullptr;
    try {
        HCHECK(hipSetDevice(ctx->device));
    } catch (const HipFail& f) {
        return set_err(ctx, ELSES_ERR_HIP, std::string(f.what) + ": " + hipGetErrorString(f.e));
    }
    return regions_create_impl(ctx, mat, n_regions, centres, radii, nullptr, tile_width, out);
}

elses_status elses_regions_create_ex(elses_ctx ctx, elses_mat mat, int32_t n_regions, const int32_t* centres,
                                     const double* radii, const uint8_t* orb_mask, int32_t tile_width,
                                     elses_regions* out) {
    if (!ctx || !mat || !out) return ELSES_ERR_INVALID_ARG;
    *out = nullptr;
    try {
        HCHECK(hipSetDevice(ctx->device));
    } catch (const HipFail& f) {
        return set_err(ctx, ELSES_ERR_HIP, std::string(f.what) + ": " + hipGetErrorString(f.e));
    }
    return regions_create_impl(ctx, mat, n_regions, centres, radii, orb_mask, tile_width, out);
}

void elses_regions_destroy(elses_regions reg) { delete reg; }

elses_status elses_regions_info(elses_regions reg, int32_t* n_cols, int32_t* n_tiles, int64_t* rows_total,
                                int64_t* useful_rows, int32_t* cols, int64_t* pat_off, int32_t* region_orbitals) {
    if (!reg) return ELSES_ERR_INVALID_ARG;
    if (n_cols) *n_cols = reg->n_cols;
    if (n_tiles) *n_tiles = reg->n_tiles;
    if (rows_total) *rows_total = reg->compact ? reg->cp.lane_rows : reg->bm->d.M;
    if (useful_rows) *useful_rows = reg->useful;
    if (cols) std::copy(reg->cols.begin(), reg->cols.end(), cols);
    if (pat_off) std::copy(reg->pat_off.begin(), reg->pat_off.end(), pat_off);
    if (region_orbitals) std::copy(reg->region_orbs.begin(), reg->region_orbs.end(), region_orbitals);
    return ELSES_OK;
}

elses_status elses_regions_solve_noalloc(elses_ctx ctx, elses_regions reg, int32_t n_shifts, const double* shifts,
                                        const double* c, const elses_opts* opts, double* x_out, double* rho_out,
                                        double* traces_out, double* col_traces_out, int32_t* iters_out,
                                        double* resid_out) {
    if (!ctx || !reg) return ELSES_ERR_INVALID_ARG;
    if (!reg->compact)
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "the allocation-free solve needs a compact region set");
    if (!c && (rho_out || traces_out || col_traces_out))
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "density outputs need the weights c");
    void* arena = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        arena = (ctx->device >= 0 && ctx->device < kMaxDevices) ? g_scratch_ptr[ctx->device] : nullptr;
    }
    if (!arena) return set_err(ctx, ELSES_ERR_HIP, "no scratch address for this device");
    return compact_solve(ctx, reg, n_shifts, shifts, c, opts, x_out, iters_out, resid_out, rho_out, traces_out,
                         col_traces_out, static_cast<char*>(arena), kNoAllocBytes);
}

elses_status elses_regions_columns(elses_regions reg, int32_t* col_region) {
    if (!reg || !col_region) return ELSES_ERR_INVALID_ARG;
    std::copy(reg->cp.col_region.begin(), reg->cp.col_region.end(), col_region);
    return ELSES_OK;
}

elses_status elses_regions_overlap_intervals(elses_regions reg, double* lo, double* hi) {
    if (!reg || !lo || !hi || !reg->compact) return ELSES_ERR_INVALID_ARG;
    for (int r = 0; r < reg->n_regions; ++r) region_interval(reg, r, lo[r], hi[r]);
    return ELSES_OK;
}

elses_status elses_regions_solve(elses_ctx ctx, elses_regions reg, int32_t n_shifts, const double* shifts,
                                 const double* c, const elses_opts* opts, double* x_out, double* rho_out,
                                 double* traces_out, double* col_traces_out, int32_t* iters_out,
                                 double* resid_out) {
    if (!ctx || !reg) return ELSES_ERR_INVALID_ARG;
    if (!c && (rho_out || traces_out || col_traces_out))
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "density outputs need the weights c");
    if (reg->compact)
        return compact_solve(ctx, reg, n_shifts, shifts, c, opts, x_out, iters_out, resid_out, rho_out, traces_out,
                             col_traces_out);
    return solve_core(ctx, reg->gm, reg->n_cols, reg->cols.data(), n_shifts, shifts, c, opts, x_out, iters_out,
                      resid_out, rho_out, traces_out, col_traces_out, reg);
}

elses_status elses_spmm32(elses_ctx ctx, elses_mat mat, int which, int32_t variant, int32_t nvec, const float* x,
                          float* y) {
    if (!ctx || !mat) return ELSES_ERR_INVALID_ARG;
    if ((which != 0 && which != 1) || nvec < 64 || nvec % 64 != 0 || !x || !y)
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "bad arguments (nvec must be a positive multiple of 64)");
    if (mat->precision != ELSES_MIXED)
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "FP32 products need a matrix created with ELSES_MIXED");
    const DevMatrix& d = mat->d;
    hipStream_t st = ctx->stream;
    PassArgs pa{};
    const char* verr = configure_pass(d, variant, nvec, pa);
    if (verr) return set_err(ctx, ELSES_ERR_INVALID_ARG, verr);
    if (pa.staged == 1 || pa.staged == 2)
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "the LDS-staged passes have no FP32 form");
    pa.vals32 = (pa.staged == 9) ? (which == 0 ? d.grp.A32 : d.grp.B32) : (which == 0 ? d.A32 : d.B32);
    pa.Xg32 = x;
    pa.Xio32 = y;
    launch_pass(PASS_PLAIN32, pa, st);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
        return set_err(ctx, ELSES_ERR_HIP, "spmm launch failed");
    return ELSES_OK;
}

elses_status elses_spmm(elses_ctx ctx, elses_mat mat, int which, int32_t variant, int32_t nvec, const double* x,
                        double* y) {
    if (!ctx || !mat) return ELSES_ERR_INVALID_ARG;
    if ((which != 0 && which != 1) || nvec < 1 || !x || !y)
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "bad arguments");
    const DevMatrix& d = mat->d;
    hipStream_t st = ctx->stream;
    if (nvec % 64 == 0) {
        PassArgs pa{};
        const char* verr = configure_pass(d, variant, nvec, pa);
        if (verr) return set_err(ctx, ELSES_ERR_INVALID_ARG, verr);
        pa.vals = (pa.staged == 9) ? (which == 0 ? d.grp.A : d.grp.B) : (which == 0 ? d.A : d.B);
        pa.Xg = x;
        pa.Xio = y;
        launch_pass(PASS_PLAIN, pa, st);
    } else {
        launch_spmm_generic(d, which == 0 ? d.A : d.B, nvec, nvec, x, y, st);
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
        return set_err(ctx, ELSES_ERR_HIP, "spmm launch failed");
    return ELSES_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Learned block SPAI of the overlap and the preconditioned overlap solve
// ---------------------------------------------------------------------------
namespace {

constexpr int kMlpIn = 40, kMlpHid = 128, kMlpOut = 16;
constexpr int64_t kOffW1 = 0, kOffb1 = kOffW1 + kMlpHid * kMlpIn, kOffW2 = kOffb1 + kMlpHid,
                  kOffb2 = kOffW2 + kMlpHid * kMlpHid, kOffW3 = kOffb2 + kMlpHid,
                  kOffb3 = kOffW3 + kMlpHid * kMlpHid, kOffW4 = kOffb3 + kMlpHid,
                  kOffb4 = kOffW4 + kMlpOut * kMlpHid, kMlpParams = kOffb4 + kMlpOut;

// Upper pairs (I <= J) of the block pattern with the ascending indices of the
// blocks (I, J) and (J, I).
struct PairList {
    std::vector<int> I, J, b, bt;
};

PairList make_pairs(const HostMatrix& h) {
    PairList P;
    for (int I = 0; I < h.n_atoms; ++I)
        for (int b = h.brow[I]; b < h.brow[I + 1]; ++b) {
            const int J = h.bcol[b];
            if (J < I) continue;
            const int* beg = h.bcol.data() + h.brow[J];
            const int* end = h.bcol.data() + h.brow[J + 1];
            const int bt = (int)(std::lower_bound(beg, end, I) - h.bcol.data());
            P.I.push_back(I);
            P.J.push_back(J);
            P.b.push_back(b);
            P.bt.push_back(bt);
        }
    return P;
}

struct DevPairs {
    int64_t n = 0;
    int *I = nullptr, *J = nullptr, *b = nullptr, *bt = nullptr;
};

DevPairs upload_pairs(DevPool& pool, const PairList& P, hipStream_t st) {
    DevPairs D;
    D.n = (int64_t)P.I.size();
    D.I = pool.get<int>(D.n);
    D.J = pool.get<int>(D.n);
    D.b = pool.get<int>(D.n);
    D.bt = pool.get<int>(D.n);
    HCHECK(hipMemcpyAsync(D.I, P.I.data(), sizeof(int) * D.n, hipMemcpyHostToDevice, st));
    HCHECK(hipMemcpyAsync(D.J, P.J.data(), sizeof(int) * D.n, hipMemcpyHostToDevice, st));
    HCHECK(hipMemcpyAsync(D.b, P.b.data(), sizeof(int) * D.n, hipMemcpyHostToDevice, st));
    HCHECK(hipMemcpyAsync(D.bt, P.bt.data(), sizeof(int) * D.n, hipMemcpyHostToDevice, st));
    return D;
}

void spai_features_dev(elses_mat mat, DevPool& pool, const DevPairs& D, float* feat, hipStream_t st) {
    const HostMatrix& h = mat->h;
    int* bcol = pool.get<int>(h.bcol.size());
    double* pos = pool.get<double>(h.pos.size());
    HCHECK(hipMemcpyAsync(bcol, h.bcol.data(), sizeof(int) * h.bcol.size(), hipMemcpyHostToDevice, st));
    HCHECK(hipMemcpyAsync(pos, h.pos.data(), sizeof(double) * h.pos.size(), hipMemcpyHostToDevice, st));
    launch_spai_features(D.n, D.I, D.J, D.b, mat->d, bcol, pos, h.box, feat, st);
}

// Workspace of one forward / backward pass over n rows.
struct MlpWork {
    float *Z1, *H1, *Z2, *H2, *Z3, *H3, *out, *gout, *G1, *G2, *G3;
    double *part, *loss;
    float* scale;
};

MlpWork mlp_work(DevPool& pool, int64_t n) {
    MlpWork w{};
    const size_t nh = (size_t)n * kMlpHid, no = (size_t)n * kMlpOut;
    w.Z1 = pool.get<float>(nh);
    w.H1 = pool.get<float>(nh);
    w.Z2 = pool.get<float>(nh);
    w.H2 = pool.get<float>(nh);
    w.Z3 = pool.get<float>(nh);
    w.H3 = pool.get<float>(nh);
    w.G1 = pool.get<float>(nh);
    w.G2 = pool.get<float>(nh);
    w.G3 = pool.get<float>(nh);
    w.out = pool.get<float>(no);
    w.gout = pool.get<float>(no);
    w.part = pool.get<double>(2 * 64);
    w.loss = pool.get<double>(1);
    w.scale = pool.get<float>(1);
    return w;
}

void mlp_forward(const float* th, int64_t n, const float* X, MlpWork& w, hipStream_t st) {
    const int N = (int)n;
    launch_gemm(N, kMlpHid, kMlpIn, X, kMlpIn, 1, th + kOffW1, 1, kMlpIn, w.Z1, kMlpHid, false, st);
    launch_bias_act(n, kMlpHid, w.Z1, th + kOffb1, w.H1, true, st);
    launch_gemm(N, kMlpHid, kMlpHid, w.H1, kMlpHid, 1, th + kOffW2, 1, kMlpHid, w.Z2, kMlpHid, false, st);
    launch_bias_act(n, kMlpHid, w.Z2, th + kOffb2, w.H2, true, st);
    launch_gemm(N, kMlpHid, kMlpHid, w.H2, kMlpHid, 1, th + kOffW3, 1, kMlpHid, w.Z3, kMlpHid, false, st);
    launch_bias_act(n, kMlpHid, w.Z3, th + kOffb3, w.H3, true, st);
    launch_gemm(N, kMlpOut, kMlpHid, w.H3, kMlpHid, 1, th + kOffW4, 1, kMlpHid, w.out, kMlpOut, false, st);
    launch_bias_act(n, kMlpOut, w.out, th + kOffb4, w.out, false, st);
}

// loss (device scalar) and gradient g of the masked mean squared error
void mlp_loss_grad(const float* th, int64_t n, const float* X, const float* T, const float* W, MlpWork& w, float* g,
                   hipStream_t st) {
    const int N = (int)n;
    mlp_forward(th, n, X, w, st);
    launch_loss(n * kMlpOut, w.out, T, W, w.gout, w.part, w.loss, w.scale, st);
    // layer 4
    launch_gemm(kMlpOut, kMlpHid, N, w.gout, 1, kMlpOut, w.H3, kMlpHid, 1, g + kOffW4, kMlpHid, false, st);
    launch_colsum(n, kMlpOut, w.gout, g + kOffb4, st);
    launch_gemm(N, kMlpHid, kMlpOut, w.gout, kMlpOut, 1, th + kOffW4, kMlpHid, 1, w.G3, kMlpHid, false, st);
    launch_gelu_back(n * kMlpHid, w.Z3, w.G3, st);
    // layer 3
    launch_gemm(kMlpHid, kMlpHid, N, w.G3, 1, kMlpHid, w.H2, kMlpHid, 1, g + kOffW3, kMlpHid, false, st);
    launch_colsum(n, kMlpHid, w.G3, g + kOffb3, st);
    launch_gemm(N, kMlpHid, kMlpHid, w.G3, kMlpHid, 1, th + kOffW3, kMlpHid, 1, w.G2, kMlpHid, false, st);
    launch_gelu_back(n * kMlpHid, w.Z2, w.G2, st);
    // layer 2
    launch_gemm(kMlpHid, kMlpHid, N, w.G2, 1, kMlpHid, w.H1, kMlpHid, 1, g + kOffW2, kMlpHid, false, st);
    launch_colsum(n, kMlpHid, w.G2, g + kOffb2, st);
    launch_gemm(N, kMlpHid, kMlpHid, w.G2, kMlpHid, 1, th + kOffW2, kMlpHid, 1, w.G1, kMlpHid, false, st);
    launch_gelu_back(n * kMlpHid, w.Z1, w.G1, st);
    // layer 1
    launch_gemm(kMlpHid, kMlpIn, N, w.G1, 1, kMlpHid, X, kMlpIn, 1, g + kOffW1, kMlpIn, false, st);
    launch_colsum(n, kMlpHid, w.G1, g + kOffb1, st);
}

elses_status hip_err(elses_ctx ctx, const HipFail& f) {
    const elses_status s = (f.e == hipErrorOutOfMemory) ? ELSES_ERR_OOM : ELSES_ERR_HIP;
    return set_err(ctx, s, std::string(f.what) + ": " + hipGetErrorString(f.e));
}

// x = p(B) s by the Richardson steps of `rich` from x_0 = 0 (direct passes).
// Returns the buffer holding x (xa or xb).
double* richardson_solve(const DevMatrix& d, const Rich& rich, int nvec, const double* s, double* xa, double* xb,
                         double* zero, hipStream_t st) {
    PassArgs pa{};
    configure_pass(d, 1, nvec, pa);
    pa.vals = d.B;
    pa.S = const_cast<double*>(s);
    pa.Xg = zero;
    pa.Xio = xa;
    pa.tau = rich.g0;
    launch_pass(PASS_STEP, pa, st);
    double* cur = xa;
    double* oth = xb;
    for (int k = 1; k < rich.d; ++k) {
        pa.Xg = cur;
        pa.Xio = oth;
        pa.tau = rich.tau[k - 1];
        launch_pass(PASS_STEP, pa, st);
        std::swap(cur, oth);
    }
    return cur;
}

}  // namespace

// Interval of the spectrum of M B (M the learned preconditioner, values in the
// internal layout): Lanczos in the B inner product, where M B is self-adjoint,
// widened like B's own interval.  M B has a positive spectrum iff M is SPD;
// returns false when the lower end is not positive.
bool mb_interval(elses_mat mat, const double* M_vals, DevPool& pool, hipStream_t st, double& lo, double& hi) {
    const DevMatrix& d = mat->d;
    const int M = d.M;

    // spectral interval of M B: Lanczos in the B inner product (M B is
    // self-adjoint there); M B has positive spectrum iff M is SPD
    double* v = pool.get<double>(M);
    double* u = pool.get<double>(M);
    double* vp = pool.get<double>(M);
    double* w = pool.get<double>(M);
    double* uw = pool.get<double>(M);
    double* junk = pool.get<double>(M);
    const int nbl = std::min(256, (M + 255) / 256);
    double* part = pool.get<double>(nbl);
    std::vector<double> hv(M), hp(nbl);
    uint64_t r = 0x9E3779B97F4A7C15ULL;
    for (int i = 0; i < M; ++i) {
        r ^= r << 13;
        r ^= r >> 7;
        r ^= r << 17;
        hv[i] = (double)(r >> 11) / 9007199254740992.0 - 0.5;
    }
    auto dotdev = [&](const double* a, const double* b) {
        launch_dot_partial(a, b, M, part, nbl, st);
        HCHECK(hipMemcpyAsync(hp.data(), part, sizeof(double) * nbl, hipMemcpyDeviceToHost, st));
        HCHECK(hipStreamSynchronize(st));
        double t = 0;
        for (double q : hp) t += q;
        return t;
    };
    HCHECK(hipMemcpyAsync(v, hv.data(), sizeof(double) * M, hipMemcpyHostToDevice, st));
    HCHECK(hipMemsetAsync(vp, 0, sizeof(double) * M, st));
    launch_spmm_generic(d, d.B, 1, 1, v, u, st);
    const double n0 = std::sqrt(dotdev(v, u));
    launch_lanczos_shift(junk, v, v, 1.0 / n0, M, st);
    launch_lanczos_shift(junk, u, u, 1.0 / n0, M, st);
    std::vector<double> ta, tb;
    double bprev = 0.0;
    const int steps = std::min(M, 60);
    for (int k = 0; k < steps; ++k) {
        launch_spmm_generic(d, M_vals, 1, 1, u, w, st);  // w = M B v
        const double al = dotdev(u, w);
        launch_lanczos_orth(w, v, vp, al, bprev, M, st);
        launch_spmm_generic(d, d.B, 1, 1, w, uw, st);
        const double bb2 = dotdev(w, uw);
        ta.push_back(al);
        if (k + 1 == steps || !(bb2 > 1e-24 * al * al)) break;
        const double bb = std::sqrt(bb2);
        tb.push_back(bb);
        launch_lanczos_shift(vp, v, w, 1.0 / bb, M, st);
        launch_lanczos_shift(junk, u, uw, 1.0 / bb, M, st);
        bprev = bb;
    }
    tb.resize(ta.size() - 1);
    const double tmin = tri_eig(ta, tb, 0), tmax = tri_eig(ta, tb, (int)ta.size() - 1);
    const double width = tmax - tmin;
    lo = tmin - 0.02 * width - 1e-3 * std::fabs(tmin);
    hi = tmax + 0.02 * width + 1e-3 * std::fabs(tmax);
    return (lo > 0.0) && std::isfinite(hi);

}

extern "C" {

elses_status elses_spai_pairs(elses_mat mat, int64_t* n_pairs, int32_t* pairs) {
    if (!mat || !n_pairs) return ELSES_ERR_INVALID_ARG;
    const PairList P = make_pairs(mat->h);
    *n_pairs = (int64_t)P.I.size();
    if (pairs)
        for (size_t p = 0; p < P.I.size(); ++p) {
            pairs[2 * p] = P.I[p];
            pairs[2 * p + 1] = P.J[p];
        }
    return ELSES_OK;
}

elses_status elses_spai_features(elses_ctx ctx, elses_mat mat, float* feat) {
    if (!ctx || !mat || !feat) return ELSES_ERR_INVALID_ARG;
    if (mat->h.pos.empty()) return set_err(ctx, ELSES_ERR_INVALID_ARG, "features need atom positions");
    hipStream_t st = ctx->stream;
    try {
        HCHECK(hipSetDevice(ctx->device));
        DevPool pool;
        const DevPairs D = upload_pairs(pool, make_pairs(mat->h), st);
        spai_features_dev(mat, pool, D, feat, st);
        HCHECK(hipGetLastError());
        HCHECK(hipStreamSynchronize(st));
    } catch (const HipFail& f) {
        return hip_err(ctx, f);
    }
    return ELSES_OK;
}

elses_status elses_spai_targets(elses_ctx ctx, elses_mat mat, float* target, float* mask) {
    if (!ctx || !mat || !target || !mask) return ELSES_ERR_INVALID_ARG;
    const HostMatrix& h = mat->h;
    const DevMatrix& d = mat->d;
    if (h.M > 65536) return set_err(ctx, ELSES_ERR_INVALID_ARG, "exact-inverse targets are for small systems");
    hipStream_t st = ctx->stream;
    try {
        HCHECK(hipSetDevice(ctx->device));
        DevPool pool;
        const DevPairs D = upload_pairs(pool, make_pairs(h), st);
        const Rich rich = richardson_plan(mat->b_lo, mat->b_hi, 1e-13);
        if (check_rich(ctx, rich, 1e-13, mat->b_lo, mat->b_hi) != ELSES_OK) return ELSES_ERR_INVALID_ARG;
        constexpr int kChunk = 1024;
        const size_t vsz = (size_t)h.M * kChunk;
        double* S = pool.get<double>(vsz);
        double* Xa = pool.get<double>(vsz);
        double* Xb = pool.get<double>(vsz);
        double* Z = pool.get<double>(vsz);
        HCHECK(hipMemsetAsync(Z, 0, sizeof(double) * vsz, st));
        // column chunks that end on atom boundaries
        int c0 = 0;
        while (c0 < h.M) {
            int c1 = c0;
            for (int I = 0; I < h.n_atoms; ++I)
                if (h.atom_off[I + 1] <= c0 + kChunk && h.atom_off[I + 1] > c1) c1 = h.atom_off[I + 1];
            const int ld = ((c1 - c0 + 63) / 64) * 64;
            launch_eye(h.M, ld, c0, S, st);
            double* X = richardson_solve(d, rich, ld, S, Xa, Xb, Z, st);
            launch_spai_targets(D.n, D.I, D.J, d.atom_off, X, ld, c0, target, mask, st);
            c0 = c1;
        }
        HCHECK(hipGetLastError());
        HCHECK(hipStreamSynchronize(st));
    } catch (const HipFail& f) {
        return hip_err(ctx, f);
    }
    return ELSES_OK;
}

elses_status elses_mlp_loss_grad(elses_ctx ctx, const float* params, int64_t n, const float* feat,
                                 const float* target, const float* mask, double* loss, float* grad) {
    if (!ctx || !params || !feat || !target || !mask || !grad || n < 1 || n > (1 << 22))
        return ELSES_ERR_INVALID_ARG;
    hipStream_t st = ctx->stream;
    try {
        HCHECK(hipSetDevice(ctx->device));
        DevPool pool;
        MlpWork w = mlp_work(pool, n);
        mlp_loss_grad(params, n, feat, target, mask, w, grad, st);
        double l = 0.0;
        HCHECK(hipMemcpyAsync(&l, w.loss, sizeof(double), hipMemcpyDeviceToHost, st));
        HCHECK(hipGetLastError());
        HCHECK(hipStreamSynchronize(st));
        if (loss) *loss = l;
    } catch (const HipFail& f) {
        return hip_err(ctx, f);
    }
    return ELSES_OK;
}

elses_status elses_spai_train(elses_ctx ctx, float* params, int64_t n, const float* feat, const float* target,
                              const float* mask, int32_t steps, int32_t batch, double lr, uint64_t seed,
                              double* loss_history) {
    if (!ctx || !params || !feat || !target || !mask || n < 1 || steps < 1 || batch < 1 || !(lr > 0.0))
        return ELSES_ERR_INVALID_ARG;
    hipStream_t st = ctx->stream;
    const int bs = (int)std::min<int64_t>(batch, n);
    try {
        HCHECK(hipSetDevice(ctx->device));
        DevPool pool;
        MlpWork w = mlp_work(pool, bs);
        float* g = pool.get<float>(kMlpParams);
        float* m = pool.get<float>(kMlpParams);
        float* v = pool.get<float>(kMlpParams);
        HCHECK(hipMemsetAsync(m, 0, sizeof(float) * kMlpParams, st));
        HCHECK(hipMemsetAsync(v, 0, sizeof(float) * kMlpParams, st));
        float* Xb = pool.get<float>((size_t)bs * kMlpIn);
        float* Tb = pool.get<float>((size_t)bs * kMlpOut);
        float* Wb = pool.get<float>((size_t)bs * kMlpOut);
        int* idx = pool.get<int>(bs);
        double* hist = pool.get<double>(steps);
        // seeded shuffles of the rows, one per epoch (splitmix64 + Fisher-Yates)
        std::vector<int> perm(n);
        for (int64_t i = 0; i < n; ++i) perm[i] = (int)i;
        uint64_t x = seed;
        auto next = [&]() {
            uint64_t z = (x += 0x9E3779B97F4A7C15ULL);
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
            return z ^ (z >> 31);
        };
        int64_t pos = n;
        std::vector<int> hidx(bs);
        for (int t = 0; t < steps; ++t) {
            for (int i = 0; i < bs; ++i) {
                if (pos >= n) {
                    for (int64_t k = n - 1; k > 0; --k) std::swap(perm[k], perm[next() % (uint64_t)(k + 1)]);
                    pos = 0;
                }
                hidx[i] = perm[pos++];
            }
            HCHECK(hipMemcpyAsync(idx, hidx.data(), sizeof(int) * bs, hipMemcpyHostToDevice, st));
            launch_gather_rows(bs, kMlpIn, idx, feat, Xb, st);
            launch_gather_rows(bs, kMlpOut, idx, target, Tb, st);
            launch_gather_rows(bs, kMlpOut, idx, mask, Wb, st);
            mlp_loss_grad(params, bs, Xb, Tb, Wb, w, g, st);
            HCHECK(hipMemcpyAsync(hist + t, w.loss, sizeof(double), hipMemcpyDeviceToDevice, st));
            launch_adam(kMlpParams, params, g, m, v, (float)lr, t + 1, st);
            // the host batch buffer is reused: wait for its upload
            HCHECK(hipStreamSynchronize(st));
        }
        if (loss_history)
            HCHECK(hipMemcpyAsync(loss_history, hist, sizeof(double) * steps, hipMemcpyDeviceToHost, st));
        HCHECK(hipGetLastError());
        HCHECK(hipStreamSynchronize(st));
    } catch (const HipFail& f) {
        return hip_err(ctx, f);
    }
    return ELSES_OK;
}

elses_status elses_spai_predict(elses_ctx ctx, const float* params, int64_t n, const float* feat, int32_t bf16,
                                float* out) {
    if (!ctx || !params || !feat || !out || n < 0) return ELSES_ERR_INVALID_ARG;
    if (n == 0) return ELSES_OK;
    if (bf16 && (reinterpret_cast<uintptr_t>(feat) & 15u))
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "BF16 inference reads feature rows as 16-byte vectors: feat must "
                                                   "be 16-byte aligned");
    hipStream_t st = ctx->stream;
    try {
        HCHECK(hipSetDevice(ctx->device));
        DevPool pool;
        if (bf16) {
            uint16_t* wb = pool.get<uint16_t>(kMlpParams);
            launch_to_bf16(kMlpParams, params, wb, st);
            launch_infer_bf16(n, wb, params, feat, out, st);
        } else {
            MlpWork w = mlp_work(pool, n);
            mlp_forward(params, n, feat, w, st);
            HCHECK(hipMemcpyAsync(out, w.out, sizeof(float) * n * kMlpOut, hipMemcpyDeviceToDevice, st));
        }
        HCHECK(hipGetLastError());
        HCHECK(hipStreamSynchronize(st));
    } catch (const HipFail& f) {
        return hip_err(ctx, f);
    }
    return ELSES_OK;
}

elses_status elses_spai_apply(elses_ctx ctx, elses_mat mat, const float* params, int32_t bf16, double* M_vals) {
    if (!ctx || !mat || !params || !M_vals) return ELSES_ERR_INVALID_ARG;
    if (mat->h.pos.empty()) return set_err(ctx, ELSES_ERR_INVALID_ARG, "features need atom positions");
    hipStream_t st = ctx->stream;
    try {
        HCHECK(hipSetDevice(ctx->device));
        DevPool pool;
        const DevPairs D = upload_pairs(pool, make_pairs(mat->h), st);
        float* feat = pool.get<float>((size_t)D.n * kMlpIn);
        float* out = pool.get<float>((size_t)D.n * kMlpOut);
        spai_features_dev(mat, pool, D, feat, st);
        if (bf16) {
            uint16_t* wb = pool.get<uint16_t>(kMlpParams);
            launch_to_bf16(kMlpParams, params, wb, st);
            launch_infer_bf16(D.n, wb, params, feat, out, st);
        } else {
            constexpr int64_t kRows = 65536;  // forward in slices to bound the workspace
            MlpWork w = mlp_work(pool, std::min<int64_t>(kRows, D.n));
            for (int64_t p0 = 0; p0 < D.n; p0 += kRows) {
                const int64_t nn = std::min<int64_t>(kRows, D.n - p0);
                mlp_forward(params, nn, feat + p0 * kMlpIn, w, st);
                HCHECK(hipMemcpyAsync(out + p0 * kMlpOut, w.out, sizeof(float) * nn * kMlpOut,
                                      hipMemcpyDeviceToDevice, st));
            }
        }
        launch_spai_assemble(D.n, D.I, D.J, D.b, D.bt, mat->d, out, M_vals, st);
        HCHECK(hipGetLastError());
        HCHECK(hipStreamSynchronize(st));
    } catch (const HipFail& f) {
        return hip_err(ctx, f);
    }
    return ELSES_OK;
}

elses_status elses_mat_set_preconditioner(elses_ctx ctx, elses_mat mat, const float* params, int32_t bf16) {
    if (!ctx || !mat) return ELSES_ERR_INVALID_ARG;
    HostMatrix& h = mat->h;
    auto drop_device_copy = [&]() {
        if (mat->M_dev) (void)hipFree(mat->M_dev);
        mat->M_dev = nullptr;
        mat->mb_spd = false;
        mat->mb_lo = mat->mb_hi = 0.0;
    };
    if (!params) {
        h.M_in.clear();
        drop_device_copy();
        return ELSES_OK;
    }
    if (h.n_orb.empty()) return set_err(ctx, ELSES_ERR_INVALID_ARG, "the preconditioner needs a caller-created matrix");
    const int64_t nnz = mat->d.nnz;
    const int nnzb = (int)h.bcol.size();
    std::vector<double> Mi(nnz);
    std::vector<int64_t> asc_voff(nnzb);
    try {
        HCHECK(hipSetDevice(ctx->device));
        DevPool pool;
        double* Mv = pool.get<double>(nnz);
        const elses_status st = elses_spai_apply(ctx, mat, params, bf16, Mv);
        if (st != ELSES_OK) return st;
        HCHECK(hipMemcpy(Mi.data(), Mv, sizeof(double) * nnz, hipMemcpyDeviceToHost));
        HCHECK(hipMemcpy(asc_voff.data(), mat->d.asc_voff, sizeof(int64_t) * nnzb, hipMemcpyDeviceToHost));
        for (int64_t e = 0; e < nnz; ++e)
            if (!std::isfinite(Mi[e])) return set_err(ctx, ELSES_ERR_INVALID_ARG, "the network produced a non-finite M");
        // the device copy for the global solves and the interval of M B, once
        drop_device_copy();
        double lo = 0.0, hi = 0.0;
        const bool spd = mb_interval(mat, Mv, pool, ctx->stream, lo, hi);
        HCHECK(hipMalloc((void**)&mat->M_dev, sizeof(double) * nnz));
        HCHECK(hipMemcpy(mat->M_dev, Mv, sizeof(double) * nnz, hipMemcpyDeviceToDevice));
        mat->mb_spd = spd;
        mat->mb_lo = lo;
        mat->mb_hi = hi;
    } catch (const HipFail& f) {
        drop_device_copy();
        return hip_err(ctx, f);
    }
    std::vector<double> Min(nnz);
    for (int b = 0; b < nnzb; ++b) {
        const int64_t len = h.in_voff[b + 1] - h.in_voff[b];
        for (int64_t e = 0; e < len; ++e) {
            const double v = Mi[asc_voff[b] + e];
            if (!std::isfinite(v)) return set_err(ctx, ELSES_ERR_INVALID_ARG, "the network produced a non-finite M");
            Min[h.in_voff[b] + e] = v;
        }
    }
    h.M_in.swap(Min);
    return ELSES_OK;
}

elses_status elses_ctx_solve_counts(elses_ctx ctx, int64_t* products, int64_t* fallbacks) {
    if (!ctx) return ELSES_ERR_INVALID_ARG;
    if (products) *products = ctx->last_products;
    if (fallbacks) *fallbacks = ctx->last_fallbacks;
    return ELSES_OK;
}

elses_status elses_overlap_solve(elses_ctx ctx, elses_mat mat, const double* M_vals, double tol, int32_t nvec,
                                 const double* s, double* x, int32_t* passes_out, double* bracket_out,
                                 int32_t* used_precond) {
    if (!ctx || !mat || !s || !x) return ELSES_ERR_INVALID_ARG;
    if (nvec < 64 || nvec % 64 != 0) return set_err(ctx, ELSES_ERR_INVALID_ARG, "nvec must be a multiple of 64");
    if (!(tol > 0.0 && tol < 1.0)) return set_err(ctx, ELSES_ERR_INVALID_ARG, "tol must be in (0, 1)");
    const DevMatrix& d = mat->d;
    const int M = d.M;
    hipStream_t st = ctx->stream;
    try {
        HCHECK(hipSetDevice(ctx->device));
        DevPool pool;
        double lo = mat->b_lo, hi = mat->b_hi;
        bool pre = M_vals != nullptr;
        if (pre && !mb_interval(mat, M_vals, pool, st, lo, hi)) {
            pre = false;  // M is not SPD: fall back to the plain overlap solve
            lo = mat->b_lo;
            hi = mat->b_hi;
        }
        if (bracket_out) {
            bracket_out[0] = lo;
            bracket_out[1] = hi;
        }
        const Rich rich = richardson_plan(lo, hi, tol);
        if (check_rich(ctx, rich, tol, lo, hi) != ELSES_OK) return ELSES_ERR_INVALID_ARG;
        const size_t vsz = (size_t)M * nvec;
        double* Z = pool.get<double>(vsz);
        double* Xa = pool.get<double>(vsz);
        double* Xb = pool.get<double>(vsz);
        HCHECK(hipMemsetAsync(Z, 0, sizeof(double) * vsz, st));
        double* res = nullptr;
        int passes = 0;
        if (!pre) {
            res = richardson_solve(d, rich, nvec, s, Xa, Xb, Z, st);
            passes = rich.d;
        } else {
            double* R = pool.get<double>(vsz);
            PassArgs pa{};
            configure_pass(d, 1, nvec, pa);
            // x_1 = g0 M s
            pa.vals = M_vals;
            pa.Xg = const_cast<double*>(s);
            pa.S = Z;
            pa.Xio = Xa;
            pa.tau = rich.g0;
            launch_pass(PASS_PSTEP, pa, st);
            double* cur = Xa;
            double* oth = Xb;
            for (int k = 1; k < rich.d; ++k) {
                pa.vals = d.B;  // r = s - B x_k
                pa.Xg = cur;
                pa.S = const_cast<double*>(s);
                pa.Xio = R;
                launch_pass(PASS_RESID, pa, st);
                pa.vals = M_vals;  // x_{k+1} = x_k + tau_k M r
                pa.Xg = R;
                pa.S = cur;
                pa.Xio = oth;
                pa.tau = rich.tau[k - 1];
                launch_pass(PASS_PSTEP, pa, st);
                std::swap(cur, oth);
            }
            res = cur;
            passes = 2 * rich.d - 1;
        }
        HCHECK(hipMemcpyAsync(x, res, sizeof(double) * vsz, hipMemcpyDeviceToDevice, st));
        HCHECK(hipGetLastError());
        HCHECK(hipStreamSynchronize(st));
        if (passes_out) *passes_out = passes;
        if (used_precond) *used_precond = pre ? 1 : 0;
    } catch (const HipFail& f) {
        return hip_err(ctx, f);
    }
    return ELSES_OK;
}

}  // extern "C"

extern "C" {

elses_status elses_autotune(elses_ctx ctx, elses_mat mat, int32_t mixed, int32_t max_slots, int32_t* variant_out,
                            int32_t* slots_out, double* ns_per_column_out) {
    if (!ctx || !mat) return ELSES_ERR_INVALID_ARG;
    if (mixed && mat->precision != ELSES_MIXED)
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "mixed tuning needs a matrix created with ELSES_MIXED");
    const int kind = mixed ? PASS_STEP32 : PASS_STEP;
    const int M = mat->d.M;
    // candidates: grouped passes with 4 / 2 / 1 waves per group and the XCD
    // placements 0, 1, 3; direct passes; slot counts up to the memory cap
    std::vector<int> variants;
    if (mat->d.grp.n > 0)
        for (int vid : {4, 5, 6})
            for (int place : {0, 1, 3}) variants.push_back(vid | (place << 4));
    variants.push_back(1 | (1 << 4));
    const int64_t cap_mem = (int64_t)(1.5 * 1024 * 1024 * 1024) / (5 * 8 * (int64_t)std::max(M, 1));
    const int cap = (int)std::min<int64_t>(max_slots > 0 ? max_slots : 2048, std::max<int64_t>(64, cap_mem));
    double best = 1e300;
    int bv = 0, bs = 0;
    for (int sl : {256, 512, 1024, 2048}) {
        if (sl > cap) continue;
        for (int v : variants) {
            double us = 0.0;
            if (elses_time_pass(ctx, mat, kind, v, sl, 10, &us) != ELSES_OK) continue;
            const double per = us * 1e3 / sl;
            if (per < best) {
                best = per;
                bv = v;
                bs = sl;
            }
        }
    }
    if (bs == 0) return set_err(ctx, ELSES_ERR_HIP, "no pass configuration could be timed");
    mat->tuned_variant[mixed ? 1 : 0] = bv;
    mat->tuned_slots[mixed ? 1 : 0] = bs;
    if (variant_out) *variant_out = bv;
    if (slots_out) *slots_out = bs;
    if (ns_per_column_out) *ns_per_column_out = best;
    return ELSES_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Observables from stored solutions: re-weighting, ICOHP, chemical potential
// ---------------------------------------------------------------------------
namespace {

struct ObsLayout {
    std::vector<int64_t> pat_off, blk_off, pbo;
    std::vector<int> blk_atom;
};

const char* obs_layout(const HostMatrix& h, int n_cols, const int32_t* cols, ObsLayout& L) {
    std::vector<int> orb_atom(h.M);
    for (int I = 0; I < h.n_atoms; ++I)
        for (int q = h.atom_off[I]; q < h.atom_off[I + 1]; ++q) orb_atom[q] = I;
    L.pat_off.assign(1, 0);
    L.blk_off.assign(1, 0);
    L.pbo.assign(1, 0);
    for (int c = 0; c < n_cols; ++c) {
        if (cols[c] < 0 || cols[c] >= h.M) return "column out of range";
        const int J = orb_atom[cols[c]];
        for (int b = h.brow[J]; b < h.brow[J + 1]; ++b) {
            const int I = h.bcol[b];
            L.blk_atom.push_back(I);
            L.pbo.push_back(L.pbo.back() + (h.atom_off[I + 1] - h.atom_off[I]));
        }
        L.blk_off.push_back((int64_t)L.blk_atom.size());
        L.pat_off.push_back(L.pbo.back());
    }
    return nullptr;
}

// Fermi weights of the midpoint rule: c_k = -(1/pi) w_k f(Re z_k)
void fermi_weights(int K, const double* shifts, const double* w, double mu, double tau, std::vector<double>& cw) {
    cw.assign(2 * K, 0.0);
    for (int k = 0; k < K; ++k) {
        const double t = (shifts[2 * k] - mu) / tau;
        const double f = t > 0 ? std::exp(-t) / (1.0 + std::exp(-t)) : 1.0 / (1.0 + std::exp(t));
        cw[2 * k] = -w[k] * f / 3.14159265358979323846;
    }
}

}  // namespace

extern "C" {

elses_status elses_pattern_blocks(elses_mat mat, int32_t n_cols, const int32_t* cols, int64_t* blk_off,
                                  int32_t* blk_atom) {
    if (!mat || n_cols < 0 || (n_cols > 0 && !cols) || !blk_off) return ELSES_ERR_INVALID_ARG;
    ObsLayout L;
    const char* e = obs_layout(mat->h, n_cols, cols, L);
    if (e) return set_err(mat->ctx, ELSES_ERR_INVALID_ARG, e);
    std::copy(L.blk_off.begin(), L.blk_off.end(), blk_off);
    if (blk_atom) std::copy(L.blk_atom.begin(), L.blk_atom.end(), blk_atom);
    return ELSES_OK;
}

elses_status elses_density_reweight(elses_ctx ctx, elses_mat mat, int32_t n_cols, const int32_t* cols,
                                    int32_t n_shifts, const double* c, const double* x, double* rho_out,
                                    double* traces_out, double* col_traces_out, double* icohp_out) {
    if (!ctx || !mat) return ELSES_ERR_INVALID_ARG;
    if (n_cols < 0 || n_shifts < 1 || !c || (n_cols > 0 && (!cols || !x)))
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "bad arguments");
    for (int k = 0; k < 2 * n_shifts; ++k)
        if (!std::isfinite(c[k])) return set_err(ctx, ELSES_ERR_INVALID_ARG, "non-finite weight");
    if (traces_out) traces_out[0] = traces_out[1] = 0.0;
    if (n_cols == 0) return ELSES_OK;
    ObsLayout L;
    const char* e = obs_layout(mat->h, n_cols, cols, L);
    if (e) return set_err(ctx, ELSES_ERR_INVALID_ARG, e);
    hipStream_t st = ctx->stream;
    const DevMatrix& d = mat->d;
    try {
        HCHECK(hipSetDevice(ctx->device));
        DevPool pool;
        const int64_t np = L.pat_off.back();
        int* d_cols = pool.get<int>(n_cols);
        int64_t* d_pat = pool.get<int64_t>(n_cols + 1);
        int* d_rows = pool.get<int>(np);
        int64_t* d_vidx = pool.get<int64_t>(np);
        int64_t* d_blk = pool.get<int64_t>(L.blk_off.size());
        int64_t* d_pbo = pool.get<int64_t>(L.pbo.size());
        double* d_cw = pool.get<double>(2 * n_shifts);
        double* rho = rho_out ? rho_out : pool.get<double>(np);
        double* ctr = col_traces_out ? col_traces_out : pool.get<double>(2 * (size_t)n_cols);
        double* tr2 = pool.get<double>(2);
        HCHECK(hipMemcpyAsync(d_cols, cols, sizeof(int) * n_cols, hipMemcpyHostToDevice, st));
        HCHECK(hipMemcpyAsync(d_pat, L.pat_off.data(), sizeof(int64_t) * L.pat_off.size(), hipMemcpyHostToDevice,
                              st));
        HCHECK(hipMemcpyAsync(d_blk, L.blk_off.data(), sizeof(int64_t) * L.blk_off.size(), hipMemcpyHostToDevice,
                              st));
        HCHECK(hipMemcpyAsync(d_pbo, L.pbo.data(), sizeof(int64_t) * L.pbo.size(), hipMemcpyHostToDevice, st));
        HCHECK(hipMemcpyAsync(d_cw, c, sizeof(double) * 2 * n_shifts, hipMemcpyHostToDevice, st));
        launch_pattern_setup(d, n_cols, d_cols, d_pat, d_rows, d_vidx, st);
        launch_reweight(n_cols, n_shifts, d_cw, d_pat, d_vidx, d_blk, d_pbo, d.B, d.A, x, rho, ctr, icohp_out, st);
        launch_sum_pairs(ctr, n_cols, tr2, st);
        double h2[2];
        HCHECK(hipMemcpyAsync(h2, tr2, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
        HCHECK(hipGetLastError());
        HCHECK(hipStreamSynchronize(st));
        if (traces_out) {
            traces_out[0] = h2[0];
            traces_out[1] = h2[1];
        }
    } catch (const HipFail& f) {
        return hip_err(ctx, f);
    }
    return ELSES_OK;
}

elses_status elses_chemical_potential(elses_ctx ctx, elses_mat mat, int32_t n_cols, const int32_t* cols,
                                      int32_t n_shifts, const double* shifts, const double* w, const double* x,
                                      double tau, double target, double mu_lo, double mu_hi, double mu_tol,
                                      double* mu_out, double* count_out) {
    if (!ctx || !mat || !shifts || !w || !mu_out) return ELSES_ERR_INVALID_ARG;
    if (!(tau > 0.0) || !(mu_hi > mu_lo) || !(mu_tol > 0.0))
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "need tau > 0, mu_hi > mu_lo, mu_tol > 0");
    std::vector<double> cw;
    double tr[2] = {0.0, 0.0};
    auto count = [&](double mu) -> elses_status {
        fermi_weights(n_shifts, shifts, w, mu, tau, cw);
        return elses_density_reweight(ctx, mat, n_cols, cols, n_shifts, cw.data(), x, nullptr, tr, nullptr,
                                      nullptr);
    };
    double lo = mu_lo, hi = mu_hi;
    elses_status s = count(lo);
    if (s != ELSES_OK) return s;
    const double n_lo = tr[0];
    if ((s = count(hi)) != ELSES_OK) return s;
    const double n_hi = tr[0];
    if (!(n_lo <= target && target <= n_hi))
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "target electron count is not bracketed by [mu_lo, mu_hi]");
    // the count tr(rho B) grows with mu: bisection
    for (int it = 0; it < 200 && hi - lo > mu_tol; ++it) {
        const double mid = 0.5 * (lo + hi);
        if ((s = count(mid)) != ELSES_OK) return s;
        if (tr[0] < target)
            lo = mid;
        else
            hi = mid;
    }
    *mu_out = 0.5 * (lo + hi);
    if ((s = count(*mu_out)) != ELSES_OK) return s;
    if (count_out) *count_out = tr[0];
    return ELSES_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Multiple Arnoldi method with analytic energy integration (Eqs. 15-18)
// ---------------------------------------------------------------------------
namespace {

constexpr int kMaChunkRows = 256;

elses_status arnoldi_core(elses_ctx ctx, elses_mat mat, const elses_regions_s* rp, int n_cols, const int32_t* cols,
                          const elses_arnoldi_opts* o_in, double* eps_out, double* wI_out, double* wB_out,
                          double* wA_out, int32_t* dim_out, double* rho_out, double* ctr_out) {
    elses_arnoldi_opts o;
    elses_arnoldi_opts_default(&o);
    if (o_in) o = *o_in;
    const int nu = o.nu;
    if (nu < 2 || nu > 48 || nu % 2 != 0) return set_err(ctx, ELSES_ERR_INVALID_ARG, "nu must be even and in [2, 48]");
    if (!std::isfinite(o.mu) || !(o.kT >= 0.0) || !std::isfinite(o.kT))
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "mu must be finite and kT >= 0");
    if (o.slots < 0 || o.slots % 64 != 0 || o.slots > 65536)
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "slots must be 0 or a multiple of 64 up to 65536");
    const double inner_tol = o.inner_tol > 0.0 ? o.inner_tol : 1e-13;
    if (!(inner_tol < 1.0)) return set_err(ctx, ELSES_ERR_INVALID_ARG, "inner_tol must be < 1");
    if (n_cols < 0) return set_err(ctx, ELSES_ERR_INVALID_ARG, "n_cols < 0");
    if (n_cols > 0 && !cols) return set_err(ctx, ELSES_ERR_INVALID_ARG, "cols is null");
    const DevMatrix& gd = mat->d;
    const DevMatrix& d = rp ? rp->bm->d : mat->d;
    const HostMatrix& h = mat->h;
    const int M = d.M;
    if (!rp) {
        std::vector<char> seen(gd.M, 0);
        for (int c = 0; c < n_cols; ++c) {
            if (cols[c] < 0 || cols[c] >= gd.M) return set_err(ctx, ELSES_ERR_INVALID_ARG, "column out of range");
            if (seen[cols[c]]) return set_err(ctx, ELSES_ERR_INVALID_ARG, "duplicate column");
            seen[cols[c]] = 1;
        }
    }
    if (n_cols == 0) return ELSES_OK;
    // lanes per vector row and segments (a global batch is one segment)
    const int Lw = rp ? rp->L : (o.slots > 0 ? o.slots : std::min(1024, ((n_cols + 63) / 64) * 64));
    const int n_seg = rp ? rp->n_tiles : 1;
    const int NS = n_seg * Lw;
    PassArgs pa{};
    const char* verr = configure_pass(d, o.variant, Lw, pa);
    if (verr) return set_err(ctx, ELSES_ERR_INVALID_ARG, verr);
    std::vector<int> slab_group, slab_tile, cs0, cs1, tco;
    if (rp) {
        const char* rerr = region_slabs(rp, pa, slab_group, slab_tile, cs0, cs1, tco);
        if (rerr) return set_err(ctx, ELSES_ERR_INVALID_ARG, rerr);
    }
    const double* valsA = (pa.staged == 9) ? d.grp.A : d.A;
    const double* valsB = (pa.staged == 9) ? d.grp.B : d.B;
    // row chunks inside segments
    std::vector<int> ch_r0, ch_r1, ch_seg, seg_ch0{0};
    for (int t = 0; t < n_seg; ++t) {
        const int r0 = rp ? rp->tile_row0[t] : 0, r1 = rp ? rp->tile_row0[t + 1] : M;
        for (int r = r0; r < r1; r += kMaChunkRows) {
            ch_r0.push_back(r);
            ch_r1.push_back(std::min(r + kMaChunkRows, r1));
            ch_seg.push_back(t);
        }
        seg_ch0.push_back((int)ch_r0.size());
    }
    const int n_ch = (int)ch_r0.size();
    const int Kmax = 4 * nu + 4;
    const Rich rich = richardson_plan(mat->b_lo, mat->b_hi, inner_tol);
    if (check_rich(ctx, rich, inner_tol, mat->b_lo, mat->b_hi) != ELSES_OK) return ELSES_ERR_INVALID_ARG;
    // pattern of each column (rows in the matrix of the passes)
    std::vector<int64_t> row_off(n_cols + 1, 0);
    if (rp) {
        row_off = rp->pat_off;
    } else {
        std::vector<int> orb_atom(gd.M);
        for (int I = 0; I < h.n_atoms; ++I)
            for (int q = h.atom_off[I]; q < h.atom_off[I + 1]; ++q) orb_atom[q] = I;
        for (int c = 0; c < n_cols; ++c) row_off[c + 1] = row_off[c] + h.atom_plen[orb_atom[cols[c]]];
    }
    const bool want_rho = rho_out != nullptr;
    hipStream_t st = ctx->stream;
    try {
        HCHECK(hipSetDevice(ctx->device));
        DevPool pool;
        const size_t plane = (size_t)M * Lw;
        double* W = pool.get<double>(plane * nu);
        double* Cd = pool.get<double>(plane * 4);  // A W_{2b-2}, A W_{2b-1}, B W_{2b-2}, B W_{2b-1}
        double* Xr = pool.get<double>(plane);      // Richardson iterate
        double* Z = pool.get<double>(plane);       // zero
        HCHECK(hipMemsetAsync(W, 0, sizeof(double) * plane * nu, st));
        HCHECK(hipMemsetAsync(Cd, 0, sizeof(double) * plane * 4, st));
        HCHECK(hipMemsetAsync(Xr, 0, sizeof(double) * plane, st));
        HCHECK(hipMemsetAsync(Z, 0, sizeof(double) * plane, st));
        double* part = pool.get<double>((size_t)n_ch * Kmax * Lw);
        double* coef = pool.get<double>((size_t)NS * Kmax);
        double* Hm = pool.get<double>((size_t)NS * nu * nu);
        double* Bm = pool.get<double>((size_t)NS * nu * nu);
        double* stt = pool.get<double>((size_t)NS * 5);
        unsigned long long* dead = pool.get<unsigned long long>(NS);
        double* gv = want_rho ? pool.get<double>((size_t)NS * nu) : nullptr;
        int* tabs = pool.get<int>(3 * (size_t)n_ch + seg_ch0.size());
        int *d_r0 = tabs, *d_r1 = tabs + n_ch, *d_seg = tabs + 2 * n_ch, *d_sc0 = tabs + 3 * n_ch;
        HCHECK(hipMemcpyAsync(d_r0, ch_r0.data(), sizeof(int) * n_ch, hipMemcpyHostToDevice, st));
        HCHECK(hipMemcpyAsync(d_r1, ch_r1.data(), sizeof(int) * n_ch, hipMemcpyHostToDevice, st));
        HCHECK(hipMemcpyAsync(d_seg, ch_seg.data(), sizeof(int) * n_ch, hipMemcpyHostToDevice, st));
        HCHECK(hipMemcpyAsync(d_sc0, seg_ch0.data(), sizeof(int) * seg_ch0.size(), hipMemcpyHostToDevice, st));
        if (rp) {
            int* d_sg = pool.get<int>(slab_group.size());
            int* d_stl = pool.get<int>(slab_tile.size());
            HCHECK(hipMemcpyAsync(d_sg, slab_group.data(), sizeof(int) * slab_group.size(), hipMemcpyHostToDevice, st));
            HCHECK(hipMemcpyAsync(d_stl, slab_tile.data(), sizeof(int) * slab_tile.size(), hipMemcpyHostToDevice, st));
            pa.slab_group = d_sg;
            pa.slab_tile = d_stl;
        }
        // column -> slot tables
        const int n_out = rp ? n_cols : std::min(n_cols, Lw);  // columns per batch
        int* slot_row = pool.get<int>(NS);
        int* slot_col = pool.get<int>(NS);
        int* col_slot = pool.get<int>(n_out);
        double* d_eps = pool.get<double>((size_t)n_out * nu);
        double* d_wI = pool.get<double>((size_t)n_out * nu);
        double* d_wB = pool.get<double>((size_t)n_out * nu);
        double* d_wA = pool.get<double>((size_t)n_out * nu);
        int* d_dim = pool.get<int>(n_out);
        double* d_ctr = pool.get<double>(2 * (size_t)n_out);
        int* d_rows = nullptr;
        int64_t* d_pat = nullptr;
        double* d_rho = nullptr;
        if (want_rho) {
            d_pat = rp ? rp->d_pat_off : pool.get<int64_t>(n_cols + 1);
            d_rows = rp ? rp->d_rows : pool.get<int>((size_t)row_off[n_cols]);
            d_rho = pool.get<double>((size_t)row_off[n_cols]);
            if (!rp) {
                int* d_cols = pool.get<int>(n_cols);
                int64_t* d_vidx = pool.get<int64_t>((size_t)row_off[n_cols]);
                HCHECK(hipMemcpyAsync(d_cols, cols, sizeof(int) * n_cols, hipMemcpyHostToDevice, st));
                HCHECK(hipMemcpyAsync(d_pat, row_off.data(), sizeof(int64_t) * (n_cols + 1), hipMemcpyHostToDevice, st));
                launch_pattern_setup(gd, n_cols, d_cols, d_pat, d_rows, d_vidx, st);
            }
        }
        auto reduce = [&](int K) { launch_ma_reduce(part, K, Lw, n_seg, d_sc0, coef, st); };
        auto book = [&](int op, int b, int nq, int K) {
            launch_ma_book(op, b, nu, nq, K, coef, Hm, Bm, stt, dead, slot_row, NS, st);
        };
        auto plain = [&](const double* vals, const double* x, double* y) {
            pa.vals = vals;
            pa.Xg = x;
            pa.Xio = y;
            launch_pass(PASS_PLAIN, pa, st);
        };
        auto Wk = [&](int k) { return W + (size_t)k * plane; };
        double* C0 = Cd;
        double* C1 = Cd + plane;
        // Sampled event timing of the Gram-Schmidt update passes (two per
        // block: both candidates minus their projections on the 2b basis
        // vectors so far), the kernel with the largest share of the time.
        struct EvList : std::vector<std::pair<hipEvent_t, hipEvent_t>> {
            ~EvList() {
                for (auto& e : *this) {
                    (void)hipEventDestroy(e.first);
                    (void)hipEventDestroy(e.second);
                }
            }
        } evs;
        double s_bytes = 0.0, s_flops = 0.0;
        int64_t n_upd = 0;
        auto update = [&](int nq, int K, int stats) {
            const bool timed = ctx->prof_stride > 0 && (n_upd++ % ctx->prof_stride) == 0;
            if (timed) {
                evs.emplace_back(nullptr, nullptr);
                HCHECK(hipEventCreate(&evs.back().first));
                HCHECK(hipEventCreate(&evs.back().second));
                HCHECK(hipEventRecord(evs.back().first, st));
            }
            launch_ma_update(2, Cd, plane, W, plane, nq, Lw, n_ch, d_r0, d_r1, d_seg, coef, K, stats, part, st);
            if (timed) {
                HCHECK(hipEventRecord(evs.back().second, st));
                // read nq basis + 2 candidate blocks, write 2 candidate blocks,
                // coefficients, partial Gram entries
                s_bytes += (double)(nq + 4) * plane * 8.0 + (double)n_ch * Lw * 2.0 * nq * 8.0 +
                           (stats ? (double)n_ch * 3 * Lw * 8.0 : 0.0);
                s_flops += 2.0 * (2.0 * nq + (stats ? 3.0 : 0.0)) * (double)plane;
            }
        };
        for (int c0 = 0; c0 < n_cols; c0 += n_out) {
            const int nb = std::min(n_out, n_cols - c0);
            std::vector<int> srow(NS, -1), scol(NS, -1), cslot(n_out, -1);
            if (rp) {
                for (int s = 0; s < NS; ++s) {
                    const int c = rp->slot_map[s];
                    if (c < 0) continue;
                    srow[s] = rp->col_row[c];
                    scol[s] = c;
                    cslot[c] = s;
                }
            } else {
                for (int c = 0; c < nb; ++c) {
                    srow[c] = cols[c0 + c];
                    scol[c] = c;
                    cslot[c] = c;
                }
            }
            HCHECK(hipMemcpyAsync(slot_row, srow.data(), sizeof(int) * NS, hipMemcpyHostToDevice, st));
            HCHECK(hipMemcpyAsync(slot_col, scol.data(), sizeof(int) * NS, hipMemcpyHostToDevice, st));
            HCHECK(hipMemcpyAsync(col_slot, cslot.data(), sizeof(int) * n_out, hipMemcpyHostToDevice, st));
            HCHECK(hipMemsetAsync(Hm, 0, sizeof(double) * NS * nu * nu, st));
            HCHECK(hipMemsetAsync(Bm, 0, sizeof(double) * NS * nu * nu, st));
            HCHECK(hipMemsetAsync(stt, 0, sizeof(double) * NS * 5, st));
            HCHECK(hipMemsetAsync(dead, 0, sizeof(unsigned long long) * NS, st));
            HCHECK(hipMemsetAsync(W, 0, sizeof(double) * plane, st));
            // block 0: W_0 = e_j, candidate u = p(B) e_j (Richardson from x = 0)
            launch_ma_unit(NS, Lw, slot_row, W, st);
            pa.vals = valsB;
            pa.S = W;
            pa.Xg = Z;
            pa.Xio = (rich.d % 2 == 1) ? C1 : Xr;
            pa.tau = rich.g0;
            launch_pass(PASS_STEP, pa, st);
            for (int k = 1; k < rich.d; ++k) {
                double* cur = const_cast<double*>(pa.Xio);
                pa.Xg = cur;
                pa.Xio = (cur == C1) ? Xr : C1;
                pa.tau = rich.tau[k - 1];
                launch_pass(PASS_STEP, pa, st);
            }
            launch_ma_dots(1, C1, plane, W, plane, 1, Lw, n_ch, d_r0, d_r1, part, 2, st);
            reduce(2);
            book(MA_BOOK_START, 0, 1, 2);
            for (int pass = 0; pass < 2; ++pass) {
                launch_ma_vec(1, C1, W, nullptr, Lw, n_ch, d_r0, d_r1, d_seg, stt + 4, 5, part, st);
                reduce(2);
                book(pass == 0 ? MA_BOOK_GAMMA : MA_BOOK_NORM1, 0, 0, 2);
            }
            launch_ma_vec(0, Wk(1), C1, C1, Lw, n_ch, d_r0, d_r1, d_seg, stt + 3, 5, part, st);
            // blocks b = 1 .. nu/2 - 1
            for (int b = 1; b < nu / 2; ++b) {
                plain(valsA, Wk(2 * b - 2), C0);
                plain(valsA, Wk(2 * b - 1), C1);
                plain(valsB, Wk(2 * b - 2), Cd + 2 * plane);
                plain(valsB, Wk(2 * b - 1), Cd + 3 * plane);
                const int nq = 2 * b;
                const int K1 = 4 * nq + 4, K2 = 2 * nq + 2;
                launch_ma_dots(4, Cd, plane, W, plane, nq, Lw, n_ch, d_r0, d_r1, part, K1, st);
                reduce(K1);
                book(MA_BOOK_FIRST, b, nq, K1);
                update(nq, K1, 0);
                launch_ma_dots(2, Cd, plane, W, plane, nq, Lw, n_ch, d_r0, d_r1, part, K2, st);
                reduce(K2);
                book(MA_BOOK_SECOND, b, nq, K2);
                update(nq, K2, 1);
                reduce(3);
                book(MA_BOOK_NORM0, b, nq, 3);
                launch_ma_vec(0, Wk(2 * b), C0, C1, Lw, n_ch, d_r0, d_r1, d_seg, stt + 2, 5, part, st);
                reduce(2);
                book(MA_BOOK_GAMMA, b, nq, 2);
                for (int pass = 0; pass < 2; ++pass) {
                    launch_ma_vec(1, C1, Wk(2 * b), nullptr, Lw, n_ch, d_r0, d_r1, d_seg, stt + 4, 5, part, st);
                    reduce(2);
                    book(pass == 0 ? MA_BOOK_GAMMA : MA_BOOK_NORM1, b, nq, 2);
                }
                launch_ma_vec(0, Wk(2 * b + 1), C1, C1, Lw, n_ch, d_r0, d_r1, d_seg, stt + 3, 5, part, st);
            }
            // the last two columns of A_r and B_r
            plain(valsA, Wk(nu - 2), C0);
            plain(valsA, Wk(nu - 1), C1);
            plain(valsB, Wk(nu - 2), Cd + 2 * plane);
            plain(valsB, Wk(nu - 1), Cd + 3 * plane);
            launch_ma_dots(4, Cd, plane, W, plane, nu, Lw, n_ch, d_r0, d_r1, part, Kmax, st);
            reduce(Kmax);
            book(MA_BOOK_LAST, nu / 2, nu, Kmax);
            launch_ma_eig(NS, nu, Hm, Bm, dead, slot_row, slot_col, W, plane, Lw, o.mu, o.kT, d_eps, d_wI, d_wB, d_wA,
                          d_dim, gv, d_ctr, st);
            if (want_rho)
                launch_ma_rho(nb, d_pat + c0, d_rows, col_slot, gv, nu, W, plane, Lw, d_rho, st);
            HCHECK(hipGetLastError());
            const size_t off = (size_t)c0 * nu, cnt = (size_t)nb * nu;
            if (eps_out) HCHECK(hipMemcpyAsync(eps_out + off, d_eps, sizeof(double) * cnt, hipMemcpyDeviceToHost, st));
            if (wI_out) HCHECK(hipMemcpyAsync(wI_out + off, d_wI, sizeof(double) * cnt, hipMemcpyDeviceToHost, st));
            if (wB_out) HCHECK(hipMemcpyAsync(wB_out + off, d_wB, sizeof(double) * cnt, hipMemcpyDeviceToHost, st));
            if (wA_out) HCHECK(hipMemcpyAsync(wA_out + off, d_wA, sizeof(double) * cnt, hipMemcpyDeviceToHost, st));
            if (dim_out) HCHECK(hipMemcpyAsync(dim_out + c0, d_dim, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
            if (ctr_out)
                HCHECK(hipMemcpyAsync(ctr_out + 2 * (size_t)c0, d_ctr, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost,
                                      st));
            HCHECK(hipStreamSynchronize(st));
        }
        if (want_rho)
            HCHECK(hipMemcpyAsync(rho_out, d_rho, sizeof(double) * (size_t)row_off[n_cols], hipMemcpyDeviceToHost, st));
        HCHECK(hipStreamSynchronize(st));
        if (!evs.empty()) {
            for (auto& e : evs) {
                float ms = 0.f;
                HCHECK(hipEventElapsedTime(&ms, e.first, e.second));
                ctx->prof_ms += ms;
            }
            ctx->prof_launches += (int64_t)evs.size();
            ctx->prof_bytes = s_bytes / (double)evs.size();
            ctx->prof_flops = s_flops / (double)evs.size();
            ctx->prof_slots = NS;
        }
    } catch (const HipFail& f) {
        return hip_err(ctx, f);
    }
    return ELSES_OK;
}

}  // namespace

extern "C" {

void elses_arnoldi_opts_default(elses_arnoldi_opts* o) {
    if (!o) return;
    o->nu = 30;
    o->variant = 0;
    o->slots = 0;
    o->inner_tol = 1e-13;
    o->mu = 0.0;
    o->kT = 0.0;
}

elses_status elses_arnoldi(elses_ctx ctx, elses_mat mat, int32_t n_cols, const int32_t* cols,
                           const elses_arnoldi_opts* o, double* eps, double* w_I, double* w_B, double* w_A,
                           int32_t* dim, double* rho_out, double* col_traces_out) {
    if (!ctx || !mat) return ELSES_ERR_INVALID_ARG;
    return arnoldi_core(ctx, mat, nullptr, n_cols, cols, o, eps, w_I, w_B, w_A, dim, rho_out, col_traces_out);
}

elses_status elses_regions_arnoldi(elses_ctx ctx, elses_regions reg, const elses_arnoldi_opts* o, double* eps,
                                   double* w_I, double* w_B, double* w_A, int32_t* dim, double* rho_out,
                                   double* col_traces_out) {
    if (!ctx || !reg) return ELSES_ERR_INVALID_ARG;
    if (reg->compact)
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "multiple Arnoldi runs on region tiles (tile_width 64 or 128)");
    return arnoldi_core(ctx, reg->gm, reg, reg->n_cols, reg->cols.data(), o, eps, w_I, w_B, w_A, dim, rho_out,
                        col_traces_out);
}

}  // extern "C"
