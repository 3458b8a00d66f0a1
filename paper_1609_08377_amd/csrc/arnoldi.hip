// Multiple Arnoldi method (paper Sec. III-B, Eqs. 15-18) on gfx950.
//
// For every column j the subspace is the direct sum of K_{nu/2}(A; e_j) and
// K_{nu/2}(A; B^{-1} e_j) (Eq. 15).  Its orthonormal basis W_0 .. W_{nu-1} is
// built two vectors at a time (block Arnoldi with the start block
// [e_j, B^{-1} e_j]): block b takes the candidates A W_{2b-2}, A W_{2b-1},
// orthogonalises them against all earlier vectors by two classical
// Gram-Schmidt passes, and then against each other.  A direction whose
// norm falls below 1e-10 of its candidate's ends its sequence (the vector is
// kept as zero).  The reduced matrices are
//   A_r = W^T A W  from the Gram-Schmidt coefficients (band of width 2, the
//                  last two columns by explicit dots), symmetrised;
//   B_r = W^T B W  from dots of the products B W_k with the basis.
// The reduced pencil A_r y = eps B_r y (Cholesky + cyclic Jacobi, one
// wavefront per column in LDS) gives the Ritz values and, with
// v_m = W y_m, the weights of the analytic energy sum (Eq. 18).
//
// Layout: like the sparse passes, a vector block is [rows][Lw] doubles with
// one column per lane; rows are split into segments (one for a global solve,
// one per region tile) and every per-column reduction runs over the rows of
// its lane's segment, in fixed-size row chunks, with a deterministic
// two-stage sum.  Per-column scalars live in [slot][...] arrays, slot =
// segment * Lw + lane.
#include "internal.h"

namespace elses {

namespace {

constexpr int kMaWaves = 4;  // waves per workgroup of the row-chunk kernels

// Partial dots of NC candidate planes with nq basis planes (q-group of up to
// 8 per grid.z) and, on q-group 0, the candidates' squared norms:
//   part[(chunk * K + c * nq + q) * Lw + lane],  part[(chunk * K + NC * nq + c) * Lw + lane].
template <int NC>
__global__ void __launch_bounds__(kMaWaves * kWave)
    ma_dots_kernel(const double* __restrict__ cand, size_t cstride, const double* __restrict__ W, size_t wstride,
                   int nq, int Lw, const int* __restrict__ ch_r0, const int* __restrict__ ch_r1,
                   double* __restrict__ part, int K) {
    constexpr int QG = 8;
    const int chunk = blockIdx.x;
    const int lane = blockIdx.y * kWave + (threadIdx.x & (kWave - 1));
    const int wave = threadIdx.x / kWave;
    const int q0 = blockIdx.z * QG;
    const int nqq = min(QG, nq - q0);
    const bool norms = blockIdx.z == 0;
    double acc[NC][QG];
    double nn[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        nn[c] = 0.0;
#pragma unroll
        for (int q = 0; q < QG; ++q) acc[c][q] = 0.0;
    }
    const int r1 = ch_r1[chunk];
    for (int r = ch_r0[chunk] + wave; r < r1; r += kMaWaves) {
        const size_t e = (size_t)r * Lw + lane;
        double x[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            x[c] = cand[c * cstride + e];
            nn[c] = fma(x[c], x[c], nn[c]);
        }
#pragma unroll
        for (int q = 0; q < QG; ++q) {
            if (q < nqq) {
                const double w = W[(size_t)(q0 + q) * wstride + e];
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[c][q] = fma(x[c], w, acc[c][q]);
            }
        }
    }
    __shared__ double red[kMaWaves][kWave];
    auto wave_sum = [&](double v) -> double {
        __syncthreads();
        red[wave][threadIdx.x & (kWave - 1)] = v;
        __syncthreads();
        double s = 0.0;
        if (wave == 0)
            for (int w = 0; w < kMaWaves; ++w) s += red[w][threadIdx.x];
        return s;
    };
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
        for (int q = 0; q < QG; ++q) {
            if (q < nqq) {
                const double s = wave_sum(acc[c][q]);
                if (wave == 0) part[((size_t)chunk * K + c * nq + q0 + q) * Lw + lane] = s;
            }
        }
        if (norms) {
            const double s = wave_sum(nn[c]);
            if (wave == 0) part[((size_t)chunk * K + NC * nq + c) * Lw + lane] = s;
        }
    }
}

// out[slot * K + k] = sum over the chunks of the slot's segment of
// part[(chunk * K + k) * Lw + lane], in chunk order.
__global__ void ma_reduce_kernel(const double* __restrict__ part, int K, int Lw, int n_seg,
                                 const int* __restrict__ seg_ch0, double* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)n_seg * K * Lw;
    if (t >= total) return;
    const int lane = (int)(t % Lw);
    const int k = (int)((t / Lw) % K);
    const int seg = (int)(t / ((int64_t)Lw * K));
    double s = 0.0;
    for (int ch = seg_ch0[seg]; ch < seg_ch0[seg + 1]; ++ch) s += part[((size_t)ch * K + k) * Lw + lane];
    out[((size_t)seg * Lw + lane) * K + k] = s;
}

// C_c -= sum_q coef[slot][c * nq + q] W_q for c < NC (coefficients with row
// stride K), then, with stats, the partial Gram entries of the updated
// candidates: part[(chunk * 3 + i) * Lw + lane] for C0.C0, C0.C1, C1.C1.
template <int NC>
__global__ void __launch_bounds__(kMaWaves * kWave)
    ma_update_kernel(double* __restrict__ cand, size_t cstride, const double* __restrict__ W, size_t wstride, int nq,
                     int Lw, const int* __restrict__ ch_r0, const int* __restrict__ ch_r1,
                     const int* __restrict__ ch_seg, const double* __restrict__ coef, int K, int stats,
                     double* __restrict__ part) {
    extern __shared__ double cf[];  // [NC * nq][kWave]
    const int chunk = blockIdx.x;
    const int l = threadIdx.x & (kWave - 1);
    const int lane = blockIdx.y * kWave + l;
    const int wave = threadIdx.x / kWave;
    const size_t slot = (size_t)ch_seg[chunk] * Lw + lane;
    for (int i = wave; i < NC * nq; i += kMaWaves) cf[i * kWave + l] = coef[slot * K + i];
    __syncthreads();
    double g00 = 0.0, g01 = 0.0, g11 = 0.0;
    const int r1 = ch_r1[chunk];
    for (int r = ch_r0[chunk] + wave; r < r1; r += kMaWaves) {
        const size_t e = (size_t)r * Lw + lane;
        double x[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) x[c] = cand[c * cstride + e];
        for (int q = 0; q < nq; ++q) {
            const double w = W[(size_t)q * wstride + e];
#pragma unroll
            for (int c = 0; c < NC; ++c) x[c] = fma(-cf[(c * nq + q) * kWave + l], w, x[c]);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) cand[c * cstride + e] = x[c];
        g00 = fma(x[0], x[0], g00);
        if constexpr (NC > 1) {
            g01 = fma(x[0], x[1], g01);
            g11 = fma(x[1], x[1], g11);
        }
    }
    if (!stats) return;
    __shared__ double red[kMaWaves][kWave];
    double g[3] = {g00, g01, g11};
    for (int i = 0; i < 3; ++i) {
        __syncthreads();
        red[wave][l] = g[i];
        __syncthreads();
        if (wave == 0) {
            double s = 0.0;
            for (int w = 0; w < kMaWaves; ++w) s += red[w][l];
            part[((size_t)chunk * 3 + i) * Lw + lane] = s;
        }
    }
}

// Two-vector element-wise steps with partial dots (part[(chunk * 2 + i) * Lw + lane]):
//   op 0 (scale): D = s[slot] * X;       p0 = D.Y
//   op 1 (axpy):  D = D - s[slot] * X;   p0 = X.D, p1 = D.D   (D updated in place)
__global__ void __launch_bounds__(kMaWaves * kWave)
    ma_vec_kernel(int op, double* __restrict__ D, const double* __restrict__ X, const double* __restrict__ Y, int Lw,
                  const int* __restrict__ ch_r0, const int* __restrict__ ch_r1, const int* __restrict__ ch_seg,
                  const double* __restrict__ s, int s_stride, double* __restrict__ part) {
    const int chunk = blockIdx.x;
    const int l = threadIdx.x & (kWave - 1);
    const int lane = blockIdx.y * kWave + l;
    const int wave = threadIdx.x / kWave;
    const size_t slot = (size_t)ch_seg[chunk] * Lw + lane;
    const double sc = s[slot * s_stride];
    double p0 = 0.0, p1 = 0.0;
    const int r1 = ch_r1[chunk];
    for (int r = ch_r0[chunk] + wave; r < r1; r += kMaWaves) {
        const size_t e = (size_t)r * Lw + lane;
        const double x = X[e];
        if (op == 0) {
            const double d = sc * x;
            D[e] = d;
            p0 = fma(d, Y[e], p0);
        } else {
            const double d = fma(-sc, x, D[e]);
            D[e] = d;
            p0 = fma(x, d, p0);
            p1 = fma(d, d, p1);
        }
    }
    __shared__ double red[kMaWaves][kWave];
    double g[2] = {p0, p1};
    for (int i = 0; i < 2; ++i) {
        __syncthreads();
        red[wave][l] = g[i];
        __syncthreads();
        if (wave == 0) {
            double t = 0.0;
            for (int w = 0; w < kMaWaves; ++w) t += red[w][l];
            part[((size_t)chunk * 2 + i) * Lw + lane] = t;
        }
    }
}

// W_0 = e_j: one 1 per live slot at the row of its column (plane zeroed before).
__global__ void ma_unit_kernel(int n_slots, int Lw, const int* __restrict__ slot_row, double* __restrict__ W0) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_slots) return;
    const int r = slot_row[s];
    if (r >= 0) W0[(size_t)r * Lw + (s % Lw)] = 1.0;
}

// Per-slot bookkeeping of the block step (one thread per slot).  H and Br
// are [slot][nu][nu] (row i, column k at i * nu + k); st holds per slot
// {norm of candidate 0, norm of candidate 1, scale 0, scale 1, gamma}, and
// dead the bit mask of vectors kept as zero.
struct MaBook {
    int op, b, nu, nq, K;
    const double* coef;  // [slot][K]
    double* H;
    double* Br;
    double* st;          // [slot][5]
    unsigned long long* dead;
    const int* slot_row;
    int n_slots;
};

// Operations (MaBookOp):
//   START   coefficients of {u} vs {W_0} (+ |u|^2): gamma = W_0.u, norm 1 = |u|
//   FIRST   first-pass coefficients of {A W_{2b-2}, A W_{2b-1}, B W_{2b-2}, B W_{2b-1}}
//   SECOND  second-pass coefficients of {A W_{2b-2}, A W_{2b-1}}
//   NORM0   Gram entries after the second pass: scale of W_{2b}
//   GAMMA   coefficient of candidate 1 on W_{2b} (adds to H when b > 0)
//   NORM1   |candidate 1| after its in-block passes: scale of W_{2b+1}
//   LAST    explicit dots of the last two columns of A_r and B_r

constexpr double kDeflate = 1e-10;

__global__ void ma_book_kernel(MaBook a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n_slots || a.slot_row[s] < 0) return;
    const double* cf = a.coef + (size_t)s * a.K;
    double* H = a.H + (size_t)s * a.nu * a.nu;
    double* Br = a.Br + (size_t)s * a.nu * a.nu;
    double* st = a.st + (size_t)s * 5;
    const int nu = a.nu, nq = a.nq, b = a.b;
    switch (a.op) {
        case MA_BOOK_START:
            st[4] = cf[0];
            st[1] = sqrt(cf[1]);
            break;
        case MA_BOOK_FIRST: {
            const int k0 = 2 * b - 2, k1 = 2 * b - 1;
            for (int i = 0; i < nq; ++i) {
                H[i * nu + k0] = cf[i];
                H[i * nu + k1] = cf[nq + i];
                Br[i * nu + k0] = cf[2 * nq + i];
                Br[i * nu + k1] = cf[3 * nq + i];
            }
            st[0] = sqrt(cf[4 * nq + 0]);
            st[1] = sqrt(cf[4 * nq + 1]);
            break;
        }
        case MA_BOOK_SECOND: {
            const int k0 = 2 * b - 2, k1 = 2 * b - 1;
            for (int i = 0; i < nq; ++i) {
                H[i * nu + k0] += cf[i];
                H[i * nu + k1] += cf[nq + i];
            }
            break;
        }
        case MA_BOOK_NORM0: {
            const double n0 = sqrt(cf[0]);
            const bool live = st[0] > 0.0 && n0 > kDeflate * st[0];
            st[2] = live ? 1.0 / n0 : 0.0;
            if (live)
                H[(2 * b) * nu + 2 * b - 2] = n0;
            else
                a.dead[s] |= 1ull << (2 * b);
            break;
        }
        case MA_BOOK_GAMMA:
            st[4] = cf[0];
            if (b > 0) H[(2 * b) * nu + 2 * b - 1] += cf[0];
            break;
        case MA_BOOK_NORM1: {
            const double n1 = sqrt(cf[1]);
            const bool live = st[1] > 0.0 && n1 > kDeflate * st[1];
            st[3] = live ? 1.0 / n1 : 0.0;
            if (!live)
                a.dead[s] |= 1ull << (2 * b + 1);
            else if (b > 0)
                H[(2 * b + 1) * nu + 2 * b - 1] = n1;
            break;
        }
        case MA_BOOK_LAST: {
            const int k0 = nu - 2, k1 = nu - 1;
            for (int i = 0; i < nu; ++i) {
                H[i * nu + k0] = cf[i];
                H[i * nu + k1] = cf[nu + i];
                Br[i * nu + k0] = cf[2 * nu + i];
                Br[i * nu + k1] = cf[3 * nu + i];
            }
            break;
        }
    }
}

__device__ __forceinline__ double ma_fermi(double e, double mu, double kT) {
    if (kT > 0.0) return 0.5 * (1.0 - tanh(0.5 * (e - mu) / kT));
    return e < mu ? 1.0 : (e > mu ? 0.0 : 0.5);
}

// Reduced generalized eigenproblem of one column per workgroup (one wave):
// compact the live basis indices, B_r = L L^T, C = L^{-1} A_r L^{-T}, cyclic
// Jacobi C = Z diag(eps) Z^T, Y = L^{-T} Z, then the weights of Eq. 18 and,
// for the Fermi function f(mu, kT), g = Y (f a) and the column traces.
struct MaEig {
    int nu;
    const double* H;
    const double* Br;
    const unsigned long long* dead;
    const int* slot_row;
    const int* slot_col;  // column index of the output arrays (-1 idle)
    const double* W;      // basis planes (for (W_i)_j)
    size_t wstride;
    int Lw;
    double mu, kT;
    double* eps;          // [col][nu]
    double* wI;
    double* wB;
    double* wA;
    int* dim;             // [col]
    double* g;            // [slot][nu] (may be null)
    double* ctr;          // [col][2] (may be null)
};

// MAXP: the largest number of rotation pairs per Jacobi step (nu / 2), a
// compile-time bound for the per-lane operand registers.
template <int MAXP>
__global__ void __launch_bounds__(kWave) ma_eig_kernel(MaEig a) {
    constexpr int kMaxPairs = MAXP;
    extern __shared__ double lds[];
    const int s = blockIdx.x;
    const int t = threadIdx.x;
    const int col = a.slot_col[s];
    if (a.slot_row[s] < 0 || col < 0) return;
    const int nu = a.nu;
    const int ldn = nu | 1;        // odd row stride: conflict-free LDS banks for row and column walks
    double* Cm = lds;              // [nu][ldn] C, then eigenvalues on the diagonal
    double* Lm = Cm + nu * ldn;    // [nu][ldn] Cholesky factor (lower)
    double* Zm = Lm + nu * ldn;    // [nu][ldn] Jacobi vectors, then Y
    double* av = Zm + nu * ldn;    // [nu] a_i = (W_i)_j over compact indices
    double* bv = av + nu;          // [nu] (W^T B e_j)_i
    double* cv = bv + nu;          // [nu] (W^T A e_j)_i
    double* rot = cv + nu;         // [0..7] scalars, [8..71] rotations, [72..135] f(eps_m) a_m
    __shared__ int idx[64];
    __shared__ int n_sh, perm[64];
    const double* H = a.H + (size_t)s * nu * nu;
    const double* Br = a.Br + (size_t)s * nu * nu;
    if (t == 0) {
        int n = 0;
        const unsigned long long dm = a.dead[s];
        for (int i = 0; i < nu; ++i)
            if (!((dm >> i) & 1ull)) idx[n++] = i;
        n_sh = n;
    }
    __syncthreads();
    const int n = n_sh;
    const int row_j = a.slot_row[s];
    const int lane = s % a.Lw;
    // load the compact matrices: A_r symmetrised, B_r from its upper triangle
    for (int e = t; e < n * n; e += kWave) {
        const int i = e / n, k = e % n;
        const int ii = idx[i], kk = idx[k];
        Cm[i * ldn + k] = 0.5 * (H[ii * nu + kk] + H[kk * nu + ii]);
        Lm[i * ldn + k] = ii <= kk ? Br[ii * nu + kk] : Br[kk * nu + ii];
    }
    if (t < n) {
        const int ii = idx[t];
        av[t] = a.W[(size_t)ii * a.wstride + (size_t)row_j * a.Lw + lane];
        bv[t] = Br[0 * nu + ii];  // W_0 = e_j: column 0 of B_r
        cv[t] = 0.5 * (H[ii * nu + 0] + H[0 * nu + ii]);
    }
    __syncthreads();
    // Cholesky B_r = L L^T in place (lower triangle of Lm)
    for (int j = 0; j < n; ++j) {
        if (t == 0) {
            double d = Lm[j * ldn + j];
            for (int k = 0; k < j; ++k) d -= Lm[j * ldn + k] * Lm[j * ldn + k];
            Lm[j * ldn + j] = sqrt(fmax(d, 1e-300));
        }
        __syncthreads();
        if (t > j && t < n) {
            double v = Lm[t * ldn + j];
            for (int k = 0; k < j; ++k) v -= Lm[t * ldn + k] * Lm[j * ldn + k];
            Lm[t * ldn + j] = v / Lm[j * ldn + j];
        }
        __syncthreads();
    }
    // X = L^{-1} A_r (thread t: column t), stored in Zm
    if (t < n) {
        for (int i = 0; i < n; ++i) {
            double v = Cm[i * ldn + t];
            for (int k = 0; k < i; ++k) v -= Lm[i * ldn + k] * Zm[k * ldn + t];
            Zm[i * ldn + t] = v / Lm[i * ldn + i];
        }
    }
    __syncthreads();
    // C = L^{-1} X^T (thread t: column t, from row t of X)
    if (t < n) {
        for (int i = 0; i < n; ++i) {
            double v = Zm[t * ldn + i];
            for (int k = 0; k < i; ++k) v -= Lm[i * ldn + k] * Cm[k * ldn + t];
            Cm[i * ldn + t] = v / Lm[i * ldn + i];
        }
    }
    __syncthreads();
    for (int e = t; e < n * n; e += kWave) {
        const int i = e / n, k = e % n;
        if (i < k) {
            const double v = 0.5 * (Cm[i * ldn + k] + Cm[k * ldn + i]);
            Cm[i * ldn + k] = v;
            Cm[k * ldn + i] = v;
        }
        Zm[i * ldn + k] = (i == k) ? 1.0 : 0.0;
    }
    __syncthreads();
    // Parallel Jacobi (round-robin ordering): each step rotates up to P/2
    // disjoint index pairs at once (P = n rounded up to even; pairs with the
    // padding index are skipped).  C <- J^T C J by a row pass and a column
    // pass, Z <- Z J.  Rotations stop below 1e-16 of the Frobenius norm of C.
    double* pc = rot + 8;       // [32] cos
    double* ps = pc + 32;       // [32] sin
    __shared__ int pp[32], pq[32];
    __shared__ int any_rot;
    if (t == 0) {
        double f2 = 0.0;
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) f2 += Cm[i * ldn + k] * Cm[i * ldn + k];
        rot[5] = 1e-16 * sqrt(f2);
    }
    __syncthreads();
    const int P = n + (n & 1);
    const int npair = P / 2;
    for (int sweep = 0; sweep < 30 && n > 1; ++sweep) {
        if (t == 0) any_rot = 0;
        __syncthreads();
        for (int step = 0; step < P - 1; ++step) {
            if (t < npair) {
                int a, b;
                if (t == 0) {
                    a = step;
                    b = P - 1;
                } else {
                    a = (step + t) % (P - 1);
                    b = (step - t + P - 1) % (P - 1);
                }
                const int p = min(a, b), q = max(a, b);
                double c = 1.0, sn = 0.0;
                if (q < n) {
                    const double apq = Cm[p * ldn + q];
                    if (fabs(apq) > rot[5]) {
                        const double app = Cm[p * ldn + p], aqq = Cm[q * ldn + q];
                        const double th = (aqq - app) / (2.0 * apq);
                        const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(tt * tt + 1.0);
                        sn = tt * c;
                        any_rot = 1;
                    }
                }
                pp[t] = p;
                pq[t] = q;
                pc[t] = c;
                ps[t] = (q < n) ? sn : 0.0;
            }
            __syncthreads();
            // The pairs of a step are disjoint, so every operand of a pass is
            // loaded before any result is stored (the loads overlap instead of
            // waiting behind each store).  The pair data are wave-uniform.
            int P_[kMaxPairs], Q_[kMaxPairs];
            double C_[kMaxPairs], S_[kMaxPairs], X_[kMaxPairs], Y_[kMaxPairs];
#pragma unroll
            for (int r = 0; r < kMaxPairs; ++r) {
                const bool on = r < npair;
                P_[r] = on ? pp[r] : 0;
                Q_[r] = on ? pq[r] : 0;
                C_[r] = on ? pc[r] : 1.0;
                S_[r] = on ? ps[r] : 0.0;
            }
            // rows p, q of C (thread t: column t)
            if (t < n) {
#pragma unroll
                for (int r = 0; r < kMaxPairs; ++r)
                    if (S_[r] != 0.0) {
                        X_[r] = Cm[P_[r] * ldn + t];
                        Y_[r] = Cm[Q_[r] * ldn + t];
                    }
#pragma unroll
                for (int r = 0; r < kMaxPairs; ++r)
                    if (S_[r] != 0.0) {
                        Cm[P_[r] * ldn + t] = C_[r] * X_[r] - S_[r] * Y_[r];
                        Cm[Q_[r] * ldn + t] = S_[r] * X_[r] + C_[r] * Y_[r];
                    }
            }
            __syncthreads();
            // columns p, q of C, then of Z (thread t: row t)
            if (t < n) {
#pragma unroll
                for (int r = 0; r < kMaxPairs; ++r)
                    if (S_[r] != 0.0) {
                        X_[r] = Cm[t * ldn + P_[r]];
                        Y_[r] = Cm[t * ldn + Q_[r]];
                    }
#pragma unroll
                for (int r = 0; r < kMaxPairs; ++r)
                    if (S_[r] != 0.0) {
                        Cm[t * ldn + P_[r]] = C_[r] * X_[r] - S_[r] * Y_[r];
                        Cm[t * ldn + Q_[r]] = S_[r] * X_[r] + C_[r] * Y_[r];
                    }
#pragma unroll
                for (int r = 0; r < kMaxPairs; ++r)
                    if (S_[r] != 0.0) {
                        X_[r] = Zm[t * ldn + P_[r]];
                        Y_[r] = Zm[t * ldn + Q_[r]];
                    }
#pragma unroll
                for (int r = 0; r < kMaxPairs; ++r)
                    if (S_[r] != 0.0) {
                        Zm[t * ldn + P_[r]] = C_[r] * X_[r] - S_[r] * Y_[r];
                        Zm[t * ldn + Q_[r]] = S_[r] * X_[r] + C_[r] * Y_[r];
                    }
            }
            __syncthreads();
        }
        if (any_rot == 0) break;
        __syncthreads();
    }
    // Y = L^{-T} Z (thread t: column t), in place
    if (t < n) {
        for (int i = n - 1; i >= 0; --i) {
            double v = Zm[i * ldn + t];
            for (int k = i + 1; k < n; ++k) v -= Lm[k * ldn + i] * Zm[k * ldn + t];
            Zm[i * ldn + t] = v / Lm[i * ldn + i];
        }
    }
    // ascending order of the eigenvalues: perm[rank] = index (ties by index)
    if (t < n) {
        const double e = Cm[t * ldn + t];
        int rank = 0;
        for (int k = 0; k < n; ++k) {
            const double f = Cm[k * ldn + k];
            rank += (f < e || (f == e && k < t)) ? 1 : 0;
        }
        perm[rank] = t;
    }
    __syncthreads();
    double fw = 0.0, trB = 0.0, trA = 0.0;
    const size_t o = (size_t)col * nu;
    if (t < nu) {
        if (t < n) {
            const int m = perm[t];
            const double e = Cm[m * ldn + m];
            double am = 0.0, bm = 0.0, cm = 0.0;
            for (int i = 0; i < n; ++i) {
                const double y = Zm[i * ldn + m];
                am = fma(av[i], y, am);
                bm = fma(bv[i], y, bm);
                cm = fma(cv[i], y, cm);
            }
            a.eps[o + t] = e;
            a.wI[o + t] = am * am;
            a.wB[o + t] = am * bm;
            a.wA[o + t] = am * cm;
            fw = ma_fermi(e, a.mu, a.kT);
            trB = fw * am * bm;
            trA = fw * am * cm;
            rot[72 + t] = fw * am;  // f(eps_m) a_m by sorted position
        } else {
            a.eps[o + t] = 0.0;
            a.wI[o + t] = 0.0;
            a.wB[o + t] = 0.0;
            a.wA[o + t] = 0.0;
        }
    }
    if (t == 0) a.dim[col] = n;
    __syncthreads();
    if (a.g && t < nu) {
        // g over the original basis indices: g_ii = sum_m Y[i][m] f(eps_m) a_m
        double v = 0.0;
        int ci = -1;
        for (int i = 0; i < n; ++i)
            if (idx[i] == t) ci = i;
        if (ci >= 0)
            for (int k = 0; k < n; ++k) v = fma(Zm[ci * ldn + perm[k]], rot[72 + k], v);
        a.g[(size_t)s * nu + t] = v;
    }
    if (a.ctr) {
        for (int off = 32; off > 0; off >>= 1) {
            trB += __shfl_down(trB, off);
            trA += __shfl_down(trA, off);
        }
        if (t == 0) {
            a.ctr[2 * (size_t)col] = trB;
            a.ctr[2 * (size_t)col + 1] = trA;
        }
    }
}

// The same eigensolve for two columns per wavefront (nu <= 32): half-wave h
// (lanes 32 h .. 32 h + 31) owns slot 2 * blockIdx.x + h and its own copy of
// the work arrays, so every instruction serves two columns.  Loop bounds that
// contain barriers use the larger of the two subspace dimensions; each half
// skips indices beyond its own.
__global__ void __launch_bounds__(kWave) ma_eig2_kernel(MaEig a, int n_slots) {
    extern __shared__ double lds2[];
    constexpr int kMaxPairs = 16;
    const int t = threadIdx.x;
    const int h = t >> 5, u = t & 31;
    const int s = 2 * blockIdx.x + h;
    const int nu = a.nu;
    const int ldn = nu | 1;
    const size_t per_half = 3 * (size_t)nu * ldn + 3 * nu + 104;
    double* Cm = lds2 + h * per_half;
    double* Lm = Cm + nu * ldn;
    double* Zm = Lm + nu * ldn;
    double* av = Zm + nu * ldn;
    double* bv = av + nu;
    double* cv = bv + nu;
    double* rot = cv + nu;      // [0..7] scalars, [8..23] cos, [24..39] sin, [40..71] f(eps_m) a_m
    double* pc = rot + 8;
    double* ps = rot + 24;
    double* fa = rot + 40;
    __shared__ int idx[2][32], perm[2][32], pp[2][16], pq[2][16], n_sh[2], any_rot[2];
    const bool valid = s < n_slots && a.slot_row[s] >= 0 && a.slot_col[s] >= 0;
    const int col = valid ? a.slot_col[s] : -1;
    const double* H = a.H + (size_t)(valid ? s : 0) * nu * nu;
    const double* Br = a.Br + (size_t)(valid ? s : 0) * nu * nu;
    if (u == 0) {
        int n = 0;
        if (valid) {
            const unsigned long long dm = a.dead[s];
            for (int i = 0; i < nu; ++i)
                if (!((dm >> i) & 1ull)) idx[h][n++] = i;
        }
        n_sh[h] = n;
    }
    __syncthreads();
    const int n = n_sh[h];
    const int nmax = max(n_sh[0], n_sh[1]);
    if (nmax == 0) return;
    const int row_j = valid ? a.slot_row[s] : 0;
    const int lane = s % a.Lw;
    for (int e = u; e < n * n; e += 32) {
        const int i = e / n, k = e % n;
        const int ii = idx[h][i], kk = idx[h][k];
        Cm[i * ldn + k] = 0.5 * (H[ii * nu + kk] + H[kk * nu + ii]);
        Lm[i * ldn + k] = ii <= kk ? Br[ii * nu + kk] : Br[kk * nu + ii];
    }
    if (u < n) {
        const int ii = idx[h][u];
        av[u] = a.W[(size_t)ii * a.wstride + (size_t)row_j * a.Lw + lane];
        bv[u] = Br[ii];
        cv[u] = 0.5 * (H[ii * nu] + H[ii]);
    }
    __syncthreads();
    // Cholesky B_r = L L^T
    for (int j = 0; j < nmax; ++j) {
        if (u == 0 && j < n) {
            double d = Lm[j * ldn + j];
            for (int k = 0; k < j; ++k) d -= Lm[j * ldn + k] * Lm[j * ldn + k];
            Lm[j * ldn + j] = sqrt(fmax(d, 1e-300));
        }
        __syncthreads();
        if (j < n && u > j && u < n) {
            double v = Lm[u * ldn + j];
            for (int k = 0; k < j; ++k) v -= Lm[u * ldn + k] * Lm[j * ldn + k];
            Lm[u * ldn + j] = v / Lm[j * ldn + j];
        }
        __syncthreads();
    }
    if (u < n)
        for (int i = 0; i < n; ++i) {
            double v = Cm[i * ldn + u];
            for (int k = 0; k < i; ++k) v -= Lm[i * ldn + k] * Zm[k * ldn + u];
            Zm[i * ldn + u] = v / Lm[i * ldn + i];
        }
    __syncthreads();
    if (u < n)
        for (int i = 0; i < n; ++i) {
            double v = Zm[u * ldn + i];
            for (int k = 0; k < i; ++k) v -= Lm[i * ldn + k] * Cm[k * ldn + u];
            Cm[i * ldn + u] = v / Lm[i * ldn + i];
        }
    __syncthreads();
    for (int e = u; e < n * n; e += 32) {
        const int i = e / n, k = e % n;
        if (i < k) {
            const double v = 0.5 * (Cm[i * ldn + k] + Cm[k * ldn + i]);
            Cm[i * ldn + k] = v;
            Cm[k * ldn + i] = v;
        }
        Zm[i * ldn + k] = (i == k) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (u == 0) {
        double f2 = 0.0;
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) f2 += Cm[i * ldn + k] * Cm[i * ldn + k];
        rot[5] = 1e-16 * sqrt(f2);
    }
    __syncthreads();
    // parallel Jacobi, round-robin pairs of the larger dimension
    const int P = nmax + (nmax & 1);
    const int npair = P / 2;
    for (int sweep = 0; sweep < 30 && nmax > 1; ++sweep) {
        if (u == 0) any_rot[h] = 0;
        __syncthreads();
        for (int step = 0; step < P - 1; ++step) {
            if (u < npair) {
                int pa_, pb_;
                if (u == 0) {
                    pa_ = step;
                    pb_ = P - 1;
                } else {
                    pa_ = (step + u) % (P - 1);
                    pb_ = (step - u + P - 1) % (P - 1);
                }
                const int p = min(pa_, pb_), q = max(pa_, pb_);
                double c = 1.0, sn = 0.0;
                if (q < n) {
                    const double apq = Cm[p * ldn + q];
                    if (fabs(apq) > rot[5]) {
                        const double app = Cm[p * ldn + p], aqq = Cm[q * ldn + q];
                        const double th = (aqq - app) / (2.0 * apq);
                        const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(tt * tt + 1.0);
                        sn = tt * c;
                        any_rot[h] = 1;
                    }
                }
                pp[h][u] = p;
                pq[h][u] = q;
                pc[u] = c;
                ps[u] = sn;
            }
            __syncthreads();
            int P_[kMaxPairs], Q_[kMaxPairs];
            double C_[kMaxPairs], S_[kMaxPairs], X_[kMaxPairs], Y_[kMaxPairs];
#pragma unroll
            for (int r = 0; r < kMaxPairs; ++r) {
                const bool on = r < npair;
                P_[r] = on ? pp[h][r] : 0;
                Q_[r] = on ? pq[h][r] : 0;
                C_[r] = on ? pc[r] : 1.0;
                S_[r] = on ? ps[r] : 0.0;
            }
            if (u < n) {
#pragma unroll
                for (int r = 0; r < kMaxPairs; ++r)
                    if (S_[r] != 0.0) {
                        X_[r] = Cm[P_[r] * ldn + u];
                        Y_[r] = Cm[Q_[r] * ldn + u];
                    }
#pragma unroll
                for (int r = 0; r < kMaxPairs; ++r)
                    if (S_[r] != 0.0) {
                        Cm[P_[r] * ldn + u] = C_[r] * X_[r] - S_[r] * Y_[r];
                        Cm[Q_[r] * ldn + u] = S_[r] * X_[r] + C_[r] * Y_[r];
                    }
            }
            __syncthreads();
            if (u < n) {
#pragma unroll
                for (int r = 0; r < kMaxPairs; ++r)
                    if (S_[r] != 0.0) {
                        X_[r] = Cm[u * ldn + P_[r]];
                        Y_[r] = Cm[u * ldn + Q_[r]];
                    }
#pragma unroll
                for (int r = 0; r < kMaxPairs; ++r)
                    if (S_[r] != 0.0) {
                        Cm[u * ldn + P_[r]] = C_[r] * X_[r] - S_[r] * Y_[r];
                        Cm[u * ldn + Q_[r]] = S_[r] * X_[r] + C_[r] * Y_[r];
                    }
#pragma unroll
                for (int r = 0; r < kMaxPairs; ++r)
                    if (S_[r] != 0.0) {
                        X_[r] = Zm[u * ldn + P_[r]];
                        Y_[r] = Zm[u * ldn + Q_[r]];
                    }
#pragma unroll
                for (int r = 0; r < kMaxPairs; ++r)
                    if (S_[r] != 0.0) {
                        Zm[u * ldn + P_[r]] = C_[r] * X_[r] - S_[r] * Y_[r];
                        Zm[u * ldn + Q_[r]] = S_[r] * X_[r] + C_[r] * Y_[r];
                    }
            }
            __syncthreads();
        }
        if (any_rot[0] == 0 && any_rot[1] == 0) break;
        __syncthreads();
    }
    // Y = L^{-T} Z
    if (u < n)
        for (int i = n - 1; i >= 0; --i) {
            double v = Zm[i * ldn + u];
            for (int k = i + 1; k < n; ++k) v -= Lm[k * ldn + i] * Zm[k * ldn + u];
            Zm[i * ldn + u] = v / Lm[i * ldn + i];
        }
    if (u < n) {
        const double e = Cm[u * ldn + u];
        int rank = 0;
        for (int k = 0; k < n; ++k) {
            const double f = Cm[k * ldn + k];
            rank += (f < e || (f == e && k < u)) ? 1 : 0;
        }
        perm[h][rank] = u;
    }
    __syncthreads();
    double trB = 0.0, trA = 0.0;
    if (valid && u < nu) {
        const size_t o = (size_t)col * nu;
        if (u < n) {
            const int m = perm[h][u];
            const double e = Cm[m * ldn + m];
            double am = 0.0, bm = 0.0, cm = 0.0;
            for (int i = 0; i < n; ++i) {
                const double y = Zm[i * ldn + m];
                am = fma(av[i], y, am);
                bm = fma(bv[i], y, bm);
                cm = fma(cv[i], y, cm);
            }
            a.eps[o + u] = e;
            a.wI[o + u] = am * am;
            a.wB[o + u] = am * bm;
            a.wA[o + u] = am * cm;
            const double fw = ma_fermi(e, a.mu, a.kT);
            trB = fw * am * bm;
            trA = fw * am * cm;
            fa[u] = fw * am;
        } else {
            a.eps[o + u] = 0.0;
            a.wI[o + u] = 0.0;
            a.wB[o + u] = 0.0;
            a.wA[o + u] = 0.0;
        }
        if (u == 0) a.dim[col] = n;
    }
    __syncthreads();
    if (valid && a.g && u < nu) {
        double v = 0.0;
        int ci = -1;
        for (int i = 0; i < n; ++i)
            if (idx[h][i] == u) ci = i;
        if (ci >= 0)
            for (int k = 0; k < n; ++k) v = fma(Zm[ci * ldn + perm[h][k]], fa[k], v);
        a.g[(size_t)s * nu + u] = v;
    }
    if (a.ctr) {
        for (int off = 16; off > 0; off >>= 1) {
            trB += __shfl_down(trB, off, 32);
            trA += __shfl_down(trA, off, 32);
        }
        if (valid && u == 0) {
            a.ctr[2 * (size_t)col] = trB;
            a.ctr[2 * (size_t)col + 1] = trA;
        }
    }
}

// rho on the column patterns: rho[p] = sum_i g[slot][i] W_i[row_p][lane]
// (pattern rows -1, outside a region, give 0).
__global__ void ma_rho_kernel(int n_cols, const int64_t* __restrict__ pat_off, const int* __restrict__ rows,
                              const int* __restrict__ col_slot, const double* __restrict__ g, int nu,
                              const double* __restrict__ W, size_t wstride, int Lw, double* __restrict__ rho) {
    const int c = blockIdx.x;
    if (c >= n_cols) return;
    const int s = col_slot[c];
    if (s < 0) return;
    const int lane = s % Lw;
    for (int64_t p = pat_off[c] + threadIdx.x; p < pat_off[c + 1]; p += blockDim.x) {
        const int r = rows[p];
        double v = 0.0;
        if (r >= 0)
            for (int i = 0; i < nu; ++i) v = fma(g[(size_t)s * nu + i], W[(size_t)i * wstride + (size_t)r * Lw + lane], v);
        rho[p] = v;
    }
}

}  // namespace

void launch_ma_dots(int nc, const double* cand, size_t cstride, const double* W, size_t wstride, int nq, int Lw,
                    int n_chunks, const int* ch_r0, const int* ch_r1, double* part, int K, hipStream_t st) {
    const dim3 grid(n_chunks, Lw / kWave, (nq + 7) / 8);
    const dim3 blk(kMaWaves * kWave);
    switch (nc) {
        case 1: hipLaunchKernelGGL(ma_dots_kernel<1>, grid, blk, 0, st, cand, cstride, W, wstride, nq, Lw, ch_r0, ch_r1, part, K); break;
        case 2: hipLaunchKernelGGL(ma_dots_kernel<2>, grid, blk, 0, st, cand, cstride, W, wstride, nq, Lw, ch_r0, ch_r1, part, K); break;
        default: hipLaunchKernelGGL(ma_dots_kernel<4>, grid, blk, 0, st, cand, cstride, W, wstride, nq, Lw, ch_r0, ch_r1, part, K); break;
    }
}

void launch_ma_reduce(const double* part, int K, int Lw, int n_seg, const int* seg_ch0, double* out, hipStream_t st) {
    const int64_t total = (int64_t)n_seg * K * Lw;
    hipLaunchKernelGGL(ma_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, part, K, Lw, n_seg,
                       seg_ch0, out);
}

void launch_ma_update(int nc, double* cand, size_t cstride, const double* W, size_t wstride, int nq, int Lw,
                      int n_chunks, const int* ch_r0, const int* ch_r1, const int* ch_seg, const double* coef, int K,
                      int stats, double* part, hipStream_t st) {
    const dim3 grid(n_chunks, Lw / kWave);
    const dim3 blk(kMaWaves * kWave);
    const size_t lds = sizeof(double) * (size_t)nc * nq * kWave;
    if (nc == 1)
        hipLaunchKernelGGL(ma_update_kernel<1>, grid, blk, lds, st, cand, cstride, W, wstride, nq, Lw, ch_r0, ch_r1,
                           ch_seg, coef, K, stats, part);
    else
        hipLaunchKernelGGL(ma_update_kernel<2>, grid, blk, lds, st, cand, cstride, W, wstride, nq, Lw, ch_r0, ch_r1,
                           ch_seg, coef, K, stats, part);
}

void launch_ma_vec(int op, double* D, const double* X, const double* Y, int Lw, int n_chunks, const int* ch_r0,
                   const int* ch_r1, const int* ch_seg, const double* s, int s_stride, double* part, hipStream_t st) {
    hipLaunchKernelGGL(ma_vec_kernel, dim3(n_chunks, Lw / kWave), dim3(kMaWaves * kWave), 0, st, op, D, X, Y, Lw,
                       ch_r0, ch_r1, ch_seg, s, s_stride, part);
}

void launch_ma_unit(int n_slots, int Lw, const int* slot_row, double* W0, hipStream_t st) {
    hipLaunchKernelGGL(ma_unit_kernel, dim3((n_slots + 255) / 256), dim3(256), 0, st, n_slots, Lw, slot_row, W0);
}

void launch_ma_book(int op, int b, int nu, int nq, int K, const double* coef, double* H, double* Br, double* stt,
                    unsigned long long* dead, const int* slot_row, int n_slots, hipStream_t st) {
    MaBook a{op, b, nu, nq, K, coef, H, Br, stt, dead, slot_row, n_slots};
    hipLaunchKernelGGL(ma_book_kernel, dim3((n_slots + 255) / 256), dim3(256), 0, st, a);
}

void launch_ma_eig(int n_slots, int nu, const double* H, const double* Br, const unsigned long long* dead,
                   const int* slot_row, const int* slot_col, const double* W, size_t wstride, int Lw, double mu,
                   double kT, double* eps, double* wI, double* wB, double* wA, int* dim, double* g, double* ctr,
                   hipStream_t st) {
    MaEig a{nu, H, Br, dead, slot_row, slot_col, W, wstride, Lw, mu, kT, eps, wI, wB, wA, dim, g, ctr};
    const size_t lds = sizeof(double) * (3 * (size_t)nu * (nu | 1) + 3 * nu + 72 + 64);
    if (nu <= 32) {
        const size_t lds2 = sizeof(double) * 2 * (3 * (size_t)nu * (nu | 1) + 3 * nu + 104);
        hipLaunchKernelGGL(ma_eig2_kernel, dim3((n_slots + 1) / 2), dim3(kWave), lds2, st, a, n_slots);
    } else {
        hipLaunchKernelGGL(ma_eig_kernel<24>, dim3(n_slots), dim3(kWave), lds, st, a);
    }
}

void launch_ma_rho(int n_cols, const int64_t* pat_off, const int* rows, const int* col_slot, const double* g, int nu,
                   const double* W, size_t wstride, int Lw, double* rho, hipStream_t st) {
    if (n_cols <= 0) return;
    hipLaunchKernelGGL(ma_rho_kernel, dim3(n_cols), dim3(128), 0, st, n_cols, pat_off, rows, col_slot, g, nu, W,
                       wstride, Lw, rho);
}

}  // namespace elses
