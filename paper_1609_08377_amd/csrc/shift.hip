// Per-column work of the shifted solver (gfx950): reductions of the fused
// dot-product partials, the multi-shift recurrences on the output rows,
// convergence, refilling of finished slots from the column queue, and the
// density-matrix assembly.
//
// The outer method is a Lanczos process for B^{-1}A in the B inner product
// started from B^{-1} e_j (paper Eqs. 13-14).  With the Lanczos scalars
// alpha_n, beta_n the Galerkin approximation of each shifted system is
// x_k = Q_n (z_k I - T_n)^{-1} beta_0 e_1.  The LU factors of z_k I - T_n give
// the short recurrences used here (per shift k):
//   eta_1 = z_k - alpha_1,                  zeta_1 = beta_0
//   eta_n = z_k - alpha_n - beta_{n-1}^2 / eta_{n-1},
//   zeta_n = (beta_{n-1} / eta_{n-1}) zeta_{n-1}
//   p_n = (q_n + beta_{n-1} p_{n-1}) / eta_n,     x_n = x_{n-1} + zeta_n p_n
// and the residual of shift k is (zeta_n / eta_n) s_n with s_n = beta_n t_{n+1}
// the Lanczos residual vector, so ||r_k|| = |zeta_n / eta_n| ||s_n||.
// Im eta_n >= Im z_k > 0, so no pivot vanishes.  Only the rows the caller
// asked for (the pattern P_j, or all rows) are carried.
#include "internal.h"

namespace elses {

__device__ __forceinline__ double block_sum(double v, double* sh) {
    // wave64 reduction with cross-lane shuffles, then across waves via LDS
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) t += sh[i];
    return t;
}

struct cd {
    double r, i;
};
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cd cinv(cd a) {
    // 1/a with scaling to avoid overflow
    const double s = fabs(a.r) >= fabs(a.i) ? a.r : a.i;
    const double ar = a.r / s, ai = a.i / s;
    const double d = (ar * ar + ai * ai) * s;
    return {ar / d, -ai / d};
}

constexpr int kShiftThreads = 256;
constexpr int kChunk = 2048;  // rows staged in LDS per chunk

__global__ __launch_bounds__(kShiftThreads) void shift_update_kernel(ShiftArgs a) {
    const int slot = blockIdx.x;
    const int t = threadIdx.x;
    const int jrow = a.slot_row[slot];
    if (jrow < 0) return;
    const int n = a.slot_n[slot];
    const int cidx = a.slot_cidx[slot];
    const int K = a.K;

    __shared__ double sh_red[16];
    __shared__ double sq[kChunk];
    __shared__ cd s_ieta[256];
    __shared__ cd s_zeta[256];
    __shared__ int s_act[256];

    const double vs = a.vs[slot], ss = a.ss[slot];

    if (n == 0) {
        // start vector c = B^{-1} e_j: beta_0 = sqrt(e_j^T B^{-1} e_j)
        const double b0 = sqrt(fmax(vs, 0.0));
        if (t == 0) {
            a.beta_prev[slot] = b0;
            a.inv_beta[slot] = 1.0 / b0;
            a.coefT[slot] = 0.0;
            a.slot_n[slot] = 1;
        }
        for (int k = t; k < K; k += kShiftThreads) {
            a.conv[(size_t)slot * K + k] = 0;
            a.res[(size_t)slot * K + k] = 1.0;
        }
        return;
    }

    const double alpha = a.alpha[slot];
    const double bprev = a.beta_prev[slot];
    const double beta = sqrt(fmax(vs, 0.0));
    const double snorm = sqrt(fmax(ss, 0.0));

    int all_conv = 1;
    for (int k = t; k < K; k += kShiftThreads) {
        const size_t sk = (size_t)slot * K + k;
        if (a.conv[sk] != 0) {
            s_act[k] = 0;
            continue;
        }
        const cd z = {a.z[2 * k], a.z[2 * k + 1]};
        cd eta, zeta;
        if (n == 1) {
            eta = {z.r - alpha, z.i};
            zeta = {bprev, 0.0};
        } else {
            const cd eo = {a.eta[2 * sk], a.eta[2 * sk + 1]};
            const cd ieo = cinv(eo);
            const cd zo = {a.zeta[2 * sk], a.zeta[2 * sk + 1]};
            zeta = cmul(zo, {bprev * ieo.r, bprev * ieo.i});
            eta = {z.r - alpha - bprev * bprev * ieo.r, z.i - bprev * bprev * ieo.i};
        }
        const cd ie = cinv(eta);
        a.eta[2 * sk] = eta.r;
        a.eta[2 * sk + 1] = eta.i;
        a.zeta[2 * sk] = zeta.r;
        a.zeta[2 * sk + 1] = zeta.i;
        const cd ratio = cmul(zeta, ie);
        const double r = sqrt(ratio.r * ratio.r + ratio.i * ratio.i) * snorm;
        a.res[sk] = r;
        s_ieta[k] = ie;
        s_zeta[k] = zeta;
        s_act[k] = 1;
        if (r <= a.tol) {
            a.conv[sk] = n;
        } else {
            all_conv = 0;
        }
    }
    const int done = __syncthreads_and(all_conv);

    // vector updates on the carried rows
    const int len = a.full ? a.M : (int)(a.row_off[cidx + 1] - a.row_off[cidx]);
    const int* rows = a.full ? nullptr : a.rows + a.row_off[cidx];
    const double qs = a.inv_beta[slot];
    const int vcol = slot % a.vld;
    double* xs = a.xs + (size_t)slot * K * a.rmax * 2;
    double* ps = a.ps + (size_t)slot * K * a.rmax * 2;
    for (int base = 0; base < len; base += kChunk) {
        const int cl = min(kChunk, len - base);
        for (int p = t; p < cl; p += kShiftThreads) {
            const int row = rows ? rows[base + p] : base + p;  // -1: outside the column's region
            sq[p] = row >= 0 ? a.Vq[(size_t)row * a.vld + vcol] * qs : 0.0;
        }
        __syncthreads();
        const int tot = K * cl;
        for (int idx = t; idx < tot; idx += kShiftThreads) {
            const int k = idx / cl;
            const int p = idx - k * cl;
            if (!s_act[k]) continue;
            const size_t e = ((size_t)k * a.rmax + base + p) * 2;
            const double q = sq[p];
            const cd ie = s_ieta[k];
            double pr, pi;
            if (n == 1) {
                pr = q * ie.r;
                pi = q * ie.i;
            } else {
                const double ur = q + bprev * ps[e], ui = bprev * ps[e + 1];
                pr = ur * ie.r - ui * ie.i;
                pi = ur * ie.i + ui * ie.r;
            }
            ps[e] = pr;
            ps[e + 1] = pi;
            const cd zt = s_zeta[k];
            double xr = (n == 1) ? 0.0 : xs[e];
            double xi = (n == 1) ? 0.0 : xs[e + 1];
            xr += zt.r * pr - zt.i * pi;
            xi += zt.r * pi + zt.i * pr;
            xs[e] = xr;
            xs[e + 1] = xi;
        }
        __syncthreads();
    }

    // Breakdown: beta_n^2 = v.s at the rounding level means the Krylov space
    // is invariant (exhausted for a small problem); the current iterates are
    // then exact for every shift and the column ends here.
    const bool breakdown = !(vs > 0.0) || !(beta > 1e-13 * (fabs(alpha) + bprev));
    const bool exhausted = (n >= a.max_outer);
    if (!done && !exhausted && !breakdown) {
        if (t == 0) {
            a.beta_prev[slot] = beta;
            a.inv_beta[slot] = 1.0 / beta;
            a.coefT[slot] = beta / bprev;
            a.slot_n[slot] = n + 1;
        }
        return;
    }

    // column finished: write outputs
    if (a.x_out) {
        double* dst = a.full ? a.x_out + (size_t)cidx * K * a.M * 2 : a.x_out + (size_t)a.row_off[cidx] * K * 2;
        const int tot = K * len;
        for (int idx = t; idx < tot; idx += kShiftThreads) {
            const int k = idx / len;
            const int p = idx - k * len;
            const size_t e = ((size_t)k * a.rmax + p) * 2;
            dst[2 * (size_t)idx] = xs[e];
            dst[2 * (size_t)idx + 1] = xs[e + 1];
        }
    }
    if (a.resid_out)
        for (int k = t; k < K; k += kShiftThreads) a.resid_out[(size_t)cidx * K + k] = a.res[(size_t)slot * K + k];
    if (a.rho_out || a.ctr_out) {
        // rho_ij = sum_k Im(c_k x_{j,k,i}) and the projected traces
        double tb = 0.0, ta = 0.0;
        for (int p = t; p < len; p += kShiftThreads) {
            double r = 0.0;
            for (int k = 0; k < K; ++k) {
                const size_t e = ((size_t)k * a.rmax + p) * 2;
                r += a.cw[2 * k] * xs[e + 1] + a.cw[2 * k + 1] * xs[e];
            }
            if (a.rho_out) a.rho_out[a.row_off[cidx] + p] = r;
            if (a.vidx) {
                const int64_t vi = a.vidx[a.row_off[cidx] + p];
                tb += r * a.Bv[vi];
                ta += r * a.Av[vi];
            }
        }
        tb = block_sum(tb, sh_red);
        ta = block_sum(ta, sh_red);
        if (t == 0 && a.ctr_out) {
            a.ctr_out[2 * (size_t)cidx] = tb;
            a.ctr_out[2 * (size_t)cidx + 1] = ta;
        }
    }
    if (t == 0) {
        if (a.iters_out) a.iters_out[cidx] = n;
        if (!done) atomicAdd(a.n_notconv, 1);
        const int nxt = atomicAdd(a.queue, 1);
        if (nxt < a.n_cols) {
            a.slot_row[slot] = a.cols[nxt];
            a.slot_cidx[slot] = nxt;
        } else {
            a.slot_row[slot] = -1;
            a.slot_cidx[slot] = -1;
        }
        a.slot_n[slot] = 0;
        a.inv_beta[slot] = 0.0;
        a.coefT[slot] = 0.0;
        atomicSub(a.remaining, 1);
        if (a.tile_live) atomicSub(a.tile_live + slot / a.vld, 1);
    }
}

void launch_shift_update(const ShiftArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(shift_update_kernel, dim3(a.ld), dim3(kShiftThreads), 0, st, a);
}

// Slots 0..n_active-1 start columns 0..n_active-1 (or the columns of
// slot_map); the rest are idle.
__global__ void slot_init_kernel(ShiftArgs a, int n_active) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.ld) return;
    const int c = a.slot_map ? a.slot_map[s] : (s < n_active ? s : -1);
    a.slot_row[s] = c >= 0 ? a.cols[c] : -1;
    a.slot_cidx[s] = c;
    a.slot_n[s] = 0;
    a.inv_beta[s] = 0.0;
    a.coefT[s] = 0.0;
    a.beta_prev[s] = 0.0;
    if (s == 0) {
        // with an explicit slot map every column has its own slot: no refill
        *a.queue = a.slot_map ? a.n_cols : n_active;
        *a.remaining = a.n_cols;
        *a.n_notconv = 0;
    }
}

void launch_slot_init(const ShiftArgs& a, int n_active, hipStream_t st) {
    hipLaunchKernelGGL(slot_init_kernel, dim3((a.ld + 255) / 256), dim3(256), 0, st, a, n_active);
}

// Pattern rows and value indices of each requested column.  Column j = (J, beta):
// rows are the orbitals of the atoms coupled to J in ascending order; the value
// index points at X_{j,i} (= X_{i,j}) inside row J's blocks.
__global__ void pattern_kernel(const int* __restrict__ atom_off, const int* __restrict__ orb_atom,
                               const int* __restrict__ brow, const int* __restrict__ asc_borb,
                               const int* __restrict__ asc_n, const int64_t* __restrict__ asc_voff, int n_cols,
                               const int* __restrict__ cols, const int64_t* __restrict__ row_off, int* rows,
                               int64_t* vidx) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cols) return;
    const int j = cols[c];
    const int J = orb_atom[j];
    const int beta = j - atom_off[J];
    int64_t o = row_off[c];
    for (int b = brow[J]; b < brow[J + 1]; ++b) {
        const int nI = asc_n[b];
        for (int al = 0; al < nI; ++al) {
            rows[o] = asc_borb[b] + al;
            if (vidx) vidx[o] = asc_voff[b] + (int64_t)beta * nI + al;  // block (J, I) is n_J x n_I
            ++o;
        }
    }
}

void launch_pattern_setup(const DevMatrix& m, int n_cols, const int* cols, const int64_t* row_off, int* rows,
                          int64_t* vidx, hipStream_t st) {
    hipLaunchKernelGGL(pattern_kernel, dim3((n_cols + 127) / 128), dim3(128), 0, st, m.atom_off, m.orb_atom,
                       m.brow, m.asc_borb, m.asc_n, m.asc_voff, n_cols, cols, row_off, rows, vidx);
}

// y[r*ld + v] = sum_c X_rc x[c*ld + v], one thread per (row, vector).
__global__ void spmm_generic_kernel(const int* __restrict__ atom_off, const int* __restrict__ orb_atom,
                                    const int* __restrict__ brow, const int* __restrict__ bsplit,
                                    const int* __restrict__ borb, const int64_t* __restrict__ voff,
                                    const double* __restrict__ vals, int M, int nvec, int ld,
                                    const double* __restrict__ x, double* __restrict__ y) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)M * nvec) return;
    const int r = (int)(gid / nvec);
    const int v = (int)(gid - (int64_t)r * nvec);
    const int I = orb_atom[r];
    const int al = r - atom_off[I];
    const int nI = atom_off[I + 1] - atom_off[I];
    const int b0 = brow[I], bs = bsplit[I], b1 = brow[I + 1];
    double s = 0.0;
    const double* vr = vals + voff[I];
    for (int b = b0; b < bs; ++b) {
        const double* vb = vr + (int64_t)(b - b0) * nI * 4 + al * 4;
        const int o = borb[b];
        for (int q = 0; q < 4; ++q) s = fma(vb[q], x[(size_t)(o + q) * ld + v], s);
    }
    const double* vh = vr + (int64_t)(bs - b0) * nI * 4;
    for (int b = bs; b < b1; ++b) s = fma(vh[(int64_t)(b - bs) * nI + al], x[(size_t)borb[b] * ld + v], s);
    y[(size_t)r * ld + v] = s;
}

void launch_spmm_generic(const DevMatrix& m, const double* vals, int nvec, int ld, const double* x, double* y,
                         hipStream_t st) {
    const int64_t n = (int64_t)m.M * nvec;
    hipLaunchKernelGGL(spmm_generic_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, m.atom_off,
                       m.orb_atom, m.brow, m.bsplit, m.borb, m.voff, vals, m.M, nvec, ld, x, y);
}

__global__ void axpby_kernel(int64_t n, double a, const double* __restrict__ x, double b,
                             const double* __restrict__ y, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double t = b * y[i];
    out[i] = (a != 0.0) ? fma(a, x[i], t) : t;
}

void launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* out, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(axpby_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a, x, b, y, out);
}

__global__ void dots2_partial_kernel(int M, int ld, int n_groups, const double* __restrict__ v,
                                     const double* __restrict__ s, double* __restrict__ part0,
                                     double* __restrict__ part1) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int g = blockIdx.y;
    if (c >= ld) return;
    const int r0 = (int)((int64_t)M * g / n_groups), r1 = (int)((int64_t)M * (g + 1) / n_groups);
    double vs = 0.0, ss = 0.0;
    for (int r = r0; r < r1; ++r) {
        const double sv = s[(size_t)r * ld + c];
        vs = fma(v[(size_t)r * ld + c], sv, vs);
        ss = fma(sv, sv, ss);
    }
    part0[(size_t)g * ld + c] = vs;
    part1[(size_t)g * ld + c] = ss;
}

void launch_dots2_partial(int M, int ld, int n_groups, const double* v, const double* s, double* part0,
                          double* part1, hipStream_t st) {
    hipLaunchKernelGGL(dots2_partial_kernel, dim3((unsigned)((ld + 255) / 256), (unsigned)n_groups), dim3(256), 0,
                       st, M, ld, n_groups, v, s, part0, part1);
}

// ||e_j - (z_k B - A) x||_2 for full-mode solutions x_full [n_cols][K][M] complex,
// one workgroup per (column, shift); FP64 arithmetic on the stored values
// (FP64, or the FP32 values of a mixed-precision matrix upcast exactly).
template <typename TV>
__global__ __launch_bounds__(256) void true_residual_kernel(
    const int* __restrict__ atom_off, const int* __restrict__ orb_atom, const int* __restrict__ brow,
    const int* __restrict__ bsplit, const int* __restrict__ borb, const int64_t* __restrict__ voff,
    const TV* __restrict__ Av, const TV* __restrict__ Bv, int M, int K,
    const int* __restrict__ cols, const double* __restrict__ z, const double* __restrict__ xf,
    double* __restrict__ res) {
    __shared__ double sh[16];
    const int ck = blockIdx.x;
    const int c = ck / K, k = ck - c * K;
    const int j = cols[c];
    const double zr = z[2 * k], zi = z[2 * k + 1];
    const double* x = xf + (size_t)ck * M * 2;
    double acc = 0.0;
    for (int r = threadIdx.x; r < M; r += blockDim.x) {
        const int I = orb_atom[r];
        const int al = r - atom_off[I];
        const int nI = atom_off[I + 1] - atom_off[I];
        const int b0 = brow[I], bs = bsplit[I], b1 = brow[I + 1];
        double bxr = 0, bxi = 0, axr = 0, axi = 0;
        const int64_t vo = voff[I];
        for (int b = b0; b < b1; ++b) {
            const int nJ = (b < bs) ? 4 : 1;
            const int64_t bo = vo + ((b < bs) ? (int64_t)(b - b0) * nI * 4
                                              : (int64_t)(bs - b0) * nI * 4 + (int64_t)(b - bs) * nI) +
                               (int64_t)al * nJ;
            const int o = borb[b];
            for (int q = 0; q < nJ; ++q) {
                const double xr = x[2 * (size_t)(o + q)], xi = x[2 * (size_t)(o + q) + 1];
                const double bv = static_cast<double>(Bv[bo + q]), av = static_cast<double>(Av[bo + q]);
                bxr = fma(bv, xr, bxr);
                bxi = fma(bv, xi, bxi);
                axr = fma(av, xr, axr);
                axi = fma(av, xi, axi);
            }
        }
        double rr = (r == j ? 1.0 : 0.0) - (zr * bxr - zi * bxi - axr);
        double ri = -(zr * bxi + zi * bxr - axi);
        acc += rr * rr + ri * ri;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) res[ck] = sqrt(acc);
}

void launch_true_residual(const DevMatrix& m, bool fp32_values, int n_cols, const int* cols, int K,
                          const double* z, const double* x_full, double* res_out, hipStream_t st) {
    if (fp32_values)
        hipLaunchKernelGGL(true_residual_kernel<float>, dim3(n_cols * K), dim3(256), 0, st, m.atom_off, m.orb_atom,
                           m.brow, m.bsplit, m.borb, m.voff, m.A32, m.B32, m.M, K, cols, z, x_full, res_out);
    else
        hipLaunchKernelGGL(true_residual_kernel<double>, dim3(n_cols * K), dim3(256), 0, st, m.atom_off, m.orb_atom,
                           m.brow, m.bsplit, m.borb, m.voff, m.A, m.B, m.M, K, cols, z, x_full, res_out);
}

// Deterministic sum of n (a, b) pairs into out2[0], out2[1] (single workgroup).
__global__ void sum_pairs_kernel(const double* __restrict__ v, int n, double* __restrict__ out2) {
    __shared__ double sh[16];
    double a = 0, b = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        a += v[2 * (size_t)i];
        b += v[2 * (size_t)i + 1];
    }
    a = block_sum(a, sh);
    b = block_sum(b, sh);
    if (threadIdx.x == 0) {
        out2[0] = a;
        out2[1] = b;
    }
}

void launch_sum_pairs(const double* v, int n, double* out2, hipStream_t st) {
    hipLaunchKernelGGL(sum_pairs_kernel, dim3(1), dim3(256), 0, st, v, n, out2);
}

// part[b] = sum_{i in block b} a_i b_i (grid-stride per block), deterministic.
__global__ void dot_partial_kernel(const double* __restrict__ x, const double* __restrict__ y, int n,
                                   double* __restrict__ part) {
    __shared__ double sh[16];
    double s = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) s = fma(x[i], y[i], s);
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void launch_dot_partial(const double* a, const double* b, int n, double* part, int nblocks, hipStream_t st) {
    hipLaunchKernelGGL(dot_partial_kernel, dim3(nblocks), dim3(256), 0, st, a, b, n, part);
}

}  // namespace elses

namespace elses {

// Re-weighting of stored pattern-mode solutions (one workgroup per column):
//   rho_ij = sum_k Im(c_k x_{j,k,i}),  i in P_j            (Eq. 12 on the shifts)
//   e_j^T rho B e_j, e_j^T rho A e_j                        (Eq. 7)
//   icohp(j, I) = sum_{alpha} rho_{(I,alpha), j} A_{j, (I,alpha)} for each atom I
//                 coupled to j's atom (the ICOHP of the paper's network
//                 analysis, before the sum over the orbitals of j's atom)
// x: column c at pat_off[c] * K complex entries laid out [K][|P_j|].  Block b
// of the pattern blocks (one per coupled atom, columns in order) covers the
// pattern entries [pbo[b], pbo[b+1]); column c owns blocks [blk_off[c],
// blk_off[c+1]).  All sums run in a fixed order.
__global__ __launch_bounds__(256) void reweight_kernel(int K, const double* __restrict__ cw,
                                                       const int64_t* __restrict__ pat_off,
                                                       const int64_t* __restrict__ vidx,
                                                       const int64_t* __restrict__ blk_off,
                                                       const int64_t* __restrict__ pbo, const double* __restrict__ Bv,
                                                       const double* __restrict__ Av, const double* __restrict__ x,
                                                       double* __restrict__ rho, double* __restrict__ ctr,
                                                       double* __restrict__ icohp) {
    __shared__ double sh[16];
    const int c = blockIdx.x;
    const int64_t p0 = pat_off[c];
    const int len = (int)(pat_off[c + 1] - p0);
    const double* xc = x + p0 * K * 2;
    double tb = 0.0, ta = 0.0;
    for (int p = threadIdx.x; p < len; p += blockDim.x) {
        double r = 0.0;
        for (int k = 0; k < K; ++k) {
            const size_t e = ((size_t)k * len + p) * 2;
            r += cw[2 * k] * xc[e + 1] + cw[2 * k + 1] * xc[e];
        }
        rho[p0 + p] = r;
        const int64_t vi = vidx[p0 + p];
        tb += r * Bv[vi];
        ta += r * Av[vi];
    }
    tb = block_sum(tb, sh);
    ta = block_sum(ta, sh);
    if (threadIdx.x == 0 && ctr) {
        ctr[2 * (size_t)c] = tb;
        ctr[2 * (size_t)c + 1] = ta;
    }
    __syncthreads();  // rho of this column visible to the whole workgroup
    if (icohp)
        for (int64_t b = blk_off[c] + threadIdx.x; b < blk_off[c + 1]; b += blockDim.x) {
            double h = 0.0;
            for (int64_t q = pbo[b]; q < pbo[b + 1]; ++q) h += rho[q] * Av[vidx[q]];
            icohp[b] = h;
        }
}

void launch_reweight(int n_cols, int K, const double* cw, const int64_t* pat_off, const int64_t* vidx,
                     const int64_t* blk_off, const int64_t* pbo, const double* Bv, const double* Av,
                     const double* x, double* rho, double* ctr, double* icohp, hipStream_t st) {
    if (n_cols == 0) return;
    hipLaunchKernelGGL(reweight_kernel, dim3(n_cols), dim3(256), 0, st, K, cw, pat_off, vidx, blk_off, pbo, Bv,
                       Av, x, rho, ctr, icohp);
}

}  // namespace elses
