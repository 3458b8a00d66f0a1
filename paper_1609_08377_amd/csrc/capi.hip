// C ABI of the gfx950 generalized shifted Krylov solver: argument checks,
// upload of the atom-block matrices, the spectral bracket of B, and the
// host loop that drives the fused passes.
//
// Solver structure (paper Sec. III: (zB - A) x = e_j for many z, Eqs. 9, 13, 14):
//  * A B-inner-product Lanczos process for B^{-1}A started from B^{-1} e_j
//    spans the shift-invariant Krylov space K_n(B^{-1}A; B^{-1}e_j), shared by
//    every shift; its vectors are real.
//  * Each Lanczos step needs one overlap solve v = B^{-1} s.  It is done with a
//    fixed-degree Chebyshev iteration on an interval enclosing the spectrum
//    of B.  Being a fixed polynomial p(B), it is linear, so the Lanczos
//    correction -alpha_n q_n can be applied after the solve (p(B) t_n = q_n
//    exactly) and the process is the exact Lanczos process of the pencil
//    (A, p(B)^{-1}); the degree is chosen so that ||I - p(B) B|| <= inner_tol.
//  * A block of `ld` columns ("slots") advances together; every pass is one
//    sparse product with the block plus the step's element-wise work.  When
//    a column has converged for all shifts its slot takes the next column.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "internal.h"

namespace elses {
void launch_lanczos_orth(double* w, const double* v, const double* u, double a, double b, int n, hipStream_t st);
void launch_lanczos_shift(double* u, double* v, const double* w, double s, int n, hipStream_t st);
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

}  // namespace

extern "C" {

const char* elses_version(void) { return "elses-gfx950 0.1"; }

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
}

elses_status elses_ctx_create(int device, void* hip_stream, elses_ctx* out) {
    if (!out) return ELSES_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return ELSES_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return ELSES_ERR_HIP;
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
    void* ptrs[] = {d.atom_off, d.orb_atom, d.brow,     d.bsplit, d.borb, d.voff, d.asc_borb,
                    d.asc_n,    d.asc_voff, d.A,        d.B,      d.A32,  d.B32};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete m;
}

elses_status elses_mat_create(elses_ctx ctx, const elses_system* sys, int precision, elses_mat* out) {
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
    } catch (const HipFail& f) {
        elses_mat_destroy(m);
        const elses_status s = (f.e == hipErrorOutOfMemory) ? ELSES_ERR_OOM : ELSES_ERR_HIP;
        return set_err(ctx, s, std::string(f.what) + ": " + hipGetErrorString(f.e));
    }
    *out = m;
    return ELSES_OK;
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

struct Cheb {
    int d = 2;
    double g0 = 0;
    std::vector<double> omega, gamma;  // steps k = 1 .. d-1
};

// Chebyshev iteration for B v = s on [lo, hi]:
//   x_1 = s / theta, x_{k+1} = x_k + rho_k rho_{k-1} (x_k - x_{k-1}) + (2 rho_k / delta)(s - B x_k)
// with theta = (hi+lo)/2, delta = (hi-lo)/2, sigma = theta/delta, rho_0 = 1/sigma,
// rho_k = 1/(2 sigma - rho_{k-1}).  After d-1 products the residual is
// T_d((theta - B)/delta) / T_d(sigma) times the initial one; d is the smallest
// degree with 1/T_d(sigma) <= tol.
Cheb chebyshev_plan(double lo, double hi, double tol) {
    Cheb c;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
    const double sigma = theta / delta;
    double t0 = 1.0, t1 = sigma;
    int d = 1;
    while (1.0 / t1 > tol && d < 400) {
        const double t2 = 2.0 * sigma * t1 - t0;
        t0 = t1;
        t1 = t2;
        ++d;
    }
    c.d = std::max(d, 2);
    c.g0 = 1.0 / theta;
    double rho_prev = 1.0 / sigma;
    for (int k = 1; k < c.d; ++k) {
        const double rho = 1.0 / (2.0 * sigma - rho_prev);
        c.omega.push_back(rho * rho_prev);
        c.gamma.push_back(2.0 * rho / delta);
        rho_prev = rho;
    }
    return c;
}

int choose_slots(int n_cols, int M, const elses_opts& o) {
    if (o.slots > 0) return o.slots;
    int ld = ((n_cols + 63) / 64) * 64;
    // keep the five working blocks of [M][ld] doubles within ~1.5 GiB and ld <= 2048
    const int64_t cap_mem = (int64_t)(1.5 * 1024 * 1024 * 1024) / (5 * 8 * (int64_t)std::max(M, 1));
    int cap = (int)std::min<int64_t>(2048, std::max<int64_t>(64, (cap_mem / 64) * 64));
    ld = std::min(ld, cap);
    if (ld > 128 && ld % 128 != 0 && ld + 64 <= cap) ld += 64;
    return std::max(ld, 64);
}

elses_status solve_core(elses_ctx ctx, elses_mat mat, int n_cols, const int32_t* cols, int K,
                        const double* shifts, const double* cw, const elses_opts* opts_in, double* x_out,
                        int32_t* iters_out, double* resid_out, double* rho_out, double* traces_out,
                        double* col_traces_out) {
    if (!ctx || !mat) return ELSES_ERR_INVALID_ARG;
    elses_opts o;
    elses_opts_default(&o);
    if (opts_in) o = *opts_in;
    const DevMatrix& d = mat->d;
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
    if (o.use_mixed) return set_err(ctx, ELSES_ERR_INVALID_ARG, "mixed precision solve not available yet");
    const bool full = (o.out_mode == ELSES_OUT_FULL);
    if (o.audit && (!full || !x_out || !resid_out))
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "audit needs ELSES_OUT_FULL with x_out and resid_out");
    if (density && full) return set_err(ctx, ELSES_ERR_INVALID_ARG, "density matrix output uses the pattern mode");
    if (n_cols > 0 && !cols) return set_err(ctx, ELSES_ERR_INVALID_ARG, "cols is null");
    {
        std::vector<char> seen(M, 0);
        for (int c = 0; c < n_cols; ++c) {
            if (cols[c] < 0 || cols[c] >= M) return set_err(ctx, ELSES_ERR_INVALID_ARG, "column out of range");
            if (seen[cols[c]]) return set_err(ctx, ELSES_ERR_INVALID_ARG, "duplicate column");
            seen[cols[c]] = 1;
        }
    }
    if (traces_out) traces_out[0] = traces_out[1] = 0.0;
    if (n_cols == 0) return ELSES_OK;

    hipStream_t st = ctx->stream;
    const int ld = choose_slots(n_cols, M, o);
    if (ld % 64 != 0) return set_err(ctx, ELSES_ERR_INVALID_ARG, "slot count must be a multiple of 64");
    const int cpl = (ld % 128 == 0) ? 2 : 1;
    const int n_tiles = ld / (64 * cpl);
    const int aps = kWavesPerBlock;  // one atom per wave
    const int n_slabs = (((d.n_atoms + aps - 1) / aps + 7) / 8) * 8;
    const int rmax = full ? M : h.pmax;
    const Cheb ch = chebyshev_plan(mat->b_lo, mat->b_hi, o.inner_tol);

    // host-side pattern offsets
    std::vector<int64_t> row_off(n_cols + 1, 0);
    {
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
        const size_t vsz = (size_t)M * ld;
        double* buf[5];
        for (int i = 0; i < 5; ++i) {
            buf[i] = pool.get<double>(vsz);
            HCHECK(hipMemsetAsync(buf[i], 0, vsz * sizeof(double), st));
        }
        double* part0 = pool.get<double>((size_t)n_slabs * ld);
        double* part1 = pool.get<double>((size_t)n_slabs * ld);
        HCHECK(hipMemsetAsync(part0, 0, sizeof(double) * n_slabs * ld, st));
        HCHECK(hipMemsetAsync(part1, 0, sizeof(double) * n_slabs * ld, st));
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
        int* d_cols = pool.get<int>(n_cols);
        int64_t* d_row_off = pool.get<int64_t>(n_cols + 1);
        int* d_rows = full ? nullptr : pool.get<int>((size_t)row_off[n_cols]);
        int64_t* d_vidx = density ? pool.get<int64_t>((size_t)row_off[n_cols]) : nullptr;
        double* d_z = pool.get<double>(2 * K);
        double* d_cw = density ? pool.get<double>(2 * K) : nullptr;
        int* counters = pool.get<int>(4);
        double* ctr = (density || col_traces_out) ? (col_traces_out ? col_traces_out : pool.get<double>(2 * (size_t)n_cols))
                                                  : nullptr;
        double* tr2 = pool.get<double>(2);
        HCHECK(hipMemsetAsync(conv, 0, sizeof(int) * ld * K, st));
        HCHECK(hipMemcpyAsync(d_cols, cols, sizeof(int) * n_cols, hipMemcpyHostToDevice, st));
        HCHECK(hipMemcpyAsync(d_row_off, row_off.data(), sizeof(int64_t) * (n_cols + 1), hipMemcpyHostToDevice, st));
        HCHECK(hipMemcpyAsync(d_z, shifts, sizeof(double) * 2 * K, hipMemcpyHostToDevice, st));
        if (density) HCHECK(hipMemcpyAsync(d_cw, cw, sizeof(double) * 2 * K, hipMemcpyHostToDevice, st));
        if (!full) launch_pattern_setup(d, n_cols, d_cols, d_row_off, d_rows, d_vidx, st);

        ShiftArgs sa{};
        sa.ld = ld;
        sa.n_slabs = n_slabs;
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
        sa.part0 = part0;
        sa.part1 = part1;
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
        sa.Bv = d.B;
        sa.Av = d.A;
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

        PassArgs pa{};
        pa.atom_off = d.atom_off;
        pa.brow = d.brow;
        pa.bsplit = d.bsplit;
        pa.borb = d.borb;
        pa.voff = d.voff;
        pa.n_atoms = d.n_atoms;
        pa.ld = ld;
        pa.n_slabs = n_slabs;
        pa.atoms_per_slab = aps;
        pa.n_tiles = n_tiles;
        pa.inv_beta = inv_beta;
        pa.coefT = coefT;
        pa.alpha = alpha;
        pa.slot_n = slot_n;
        pa.slot_row = slot_row;
        pa.part0 = part0;
        pa.part1 = part1;
        pa.g0 = ch.g0;

        HCHECK(hipHostMalloc((void**)&h_rem, sizeof(int) * 4, hipHostMallocDefault));
        HCHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        double* Vq = buf[0];
        double* Xa = buf[1];
        double* Xb = buf[2];
        double* Tp = buf[3];
        double* Tn = buf[4];
        const int poll = 8;
        const int64_t generations = (n_cols + ld - 1) / ld + 1;
        const int64_t cap = (int64_t)o.max_outer * generations + 64;
        bool pending = false;
        int64_t it = 0;
        // sampled event timing of one Chebyshev pass per `prof_stride` outer iterations
        struct EvPair {
            hipEvent_t a = nullptr, b = nullptr;
            bool busy = false;
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
                    ctx->prof_launches += 1;
                    p.busy = false;
                }
        };
        if (!prof.empty()) {
            ctx->prof_bytes = (double)d.nnz * 8.0 + (double)d.nnzb * 4.0 + (double)d.n_atoms * 20.0 +
                              4.0 * (double)M * ld * 8.0;
            ctx->prof_flops = 2.0 * (double)d.nnz * ld + 6.0 * (double)M * ld;
            ctx->prof_slots = ld;
        }
        for (;;) {
            // w = A q_n, s' = w - beta t_{n-1}, alpha partials, x_1
            pa.vals = d.A;
            pa.Xg = Vq;
            pa.Xio = Xa;
            pa.S = Tp;
            pa.Vq = Vq;
            launch_pass(PASS_LANCZOS_A, pa, st);
            launch_alpha_reduce(part0, n_slabs, ld, slot_n, slot_row, alpha, st);
            // overlap solve by Chebyshev steps
            double* xcur = Xa;
            double* xoth = Xb;
            pa.vals = d.B;
            for (int k = 1; k < ch.d; ++k) {
                pa.Xg = xcur;
                pa.Xio = xoth;
                pa.omega = ch.omega[k - 1];
                pa.gamma = ch.gamma[k - 1];
                pa.has_prev = (k >= 2) ? 1 : 0;
                pa.Tn = Tn;
                EvPair* tp = nullptr;
                if (!prof.empty() && k == 2 && k < ch.d - 1 && it % ctx->prof_stride == 0)
                    for (auto& p : prof)
                        if (!p.busy) {
                            tp = &p;
                            break;
                        }
                if (tp) HCHECK(hipEventRecord(tp->a, st));
                launch_pass(k == ch.d - 1 ? PASS_CHEB_LAST : PASS_CHEB, pa, st);
                if (tp) {
                    HCHECK(hipEventRecord(tp->b, st));
                    tp->busy = true;
                }
                std::swap(xcur, xoth);
            }
            // multi-shift recurrences, convergence, slot refill
            sa.Vq = Vq;
            launch_shift_update(sa, st);
            HCHECK(hipGetLastError());
            // rotate buffers
            double* oldV = Vq;
            Vq = xcur;
            Xa = oldV;
            Xb = xoth;
            std::swap(Tp, Tn);
            ++it;
            if (it % poll == 0) {
                if (pending) {
                    HCHECK(hipEventSynchronize(ev));
                    harvest();
                    if (h_rem[0] == 0) break;
                }
                HCHECK(hipMemcpyAsync(h_rem, sa.remaining, sizeof(int), hipMemcpyDeviceToHost, st));
                HCHECK(hipEventRecord(ev, st));
                pending = true;
            }
            if (it > cap) throw HipFail{hipErrorUnknown, "solver loop did not terminate"};
        }
        if (o.audit) launch_true_residual(d, n_cols, d_cols, K, d_z, x_out, resid_out, st);
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
        ctx->total_passes += it * ch.d;
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

elses_status elses_spmm(elses_ctx ctx, elses_mat mat, int which, int32_t nvec, const double* x, double* y) {
    if (!ctx || !mat) return ELSES_ERR_INVALID_ARG;
    if ((which != 0 && which != 1) || nvec < 1 || !x || !y)
        return set_err(ctx, ELSES_ERR_INVALID_ARG, "bad arguments");
    const DevMatrix& d = mat->d;
    hipStream_t st = ctx->stream;
    const double* vals = which == 0 ? d.A : d.B;
    if (nvec % 64 == 0) {
        PassArgs pa{};
        pa.atom_off = d.atom_off;
        pa.brow = d.brow;
        pa.bsplit = d.bsplit;
        pa.borb = d.borb;
        pa.voff = d.voff;
        pa.vals = vals;
        pa.n_atoms = d.n_atoms;
        pa.ld = nvec;
        pa.atoms_per_slab = kWavesPerBlock;
        pa.n_slabs = (((d.n_atoms + kWavesPerBlock - 1) / kWavesPerBlock + 7) / 8) * 8;
        const int cpl = (nvec % 128 == 0) ? 2 : 1;
        pa.n_tiles = nvec / (64 * cpl);
        pa.Xg = x;
        pa.Xio = y;
        launch_pass(PASS_PLAIN, pa, st);
    } else {
        launch_spmm_generic(d, vals, nvec, nvec, x, y, st);
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
        return set_err(ctx, ELSES_ERR_HIP, "spmm launch failed");
    return ELSES_OK;
}

}  // extern "C"
