// Fused sparse vector passes over the atom-block matrices (gfx950).
//
// Every pass multiplies one sparse matrix (A or B) with a block of right-hand
// sides stored [M][ld] (ld = slots, one right-hand side per lane), and fuses
// the element-wise work of one step of the solver into the epilogue, so the
// vectors cross HBM as few times as possible:
//
//   PASS_LANCZOS_A  w = A q_n; s' = w - beta_{n-1} t_{n-1}; partial q_n.s';
//                   x_1 = g0 s' (first overlap-solve iterate).  Slots at
//                   n = 0 take s' = e_j instead (start vector B^{-1} e_j).
//   PASS_CHEB       one Chebyshev step of the overlap solve B v = s:
//                   x_{k+1} = x_k + omega (x_k - x_{k-1}) + gamma (s - B x_k)
//   PASS_CHEB_LAST  the last step, then the deferred Lanczos correction
//                   v = x - alpha_n q_n, s = s' - alpha_n t_n, and partial
//                   dots v.s and s.s (beta_n^2 and ||s||^2).
//   PASS_PLAIN      y = X x.
//
// Matrix values are identical for all lanes of a wave, so they are read
// through the scalar unit; each lane streams its own right-hand side.
#include "internal.h"

namespace elses {

template <int NI, int CPL>
__device__ __forceinline__ void row_product(int I, int ld, int c0, const double* __restrict__ Xg,
                                            const int* __restrict__ brow, const int* __restrict__ bsplit,
                                            const int* __restrict__ borb, const int64_t* __restrict__ voff,
                                            const double* __restrict__ vals, double (&acc)[NI][CPL]) {
#pragma unroll
    for (int a = 0; a < NI; ++a)
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[a][c] = 0.0;
    const int b0 = brow[I], bs = bsplit[I], b1 = brow[I + 1];
    const double* __restrict__ v = vals + voff[I];
    // 4-orbital neighbours
#pragma unroll 2
    for (int b = b0; b < bs; ++b) {
        const int o = borb[b];
        const double* __restrict__ xr = Xg + (size_t)o * ld + c0;
        double x[4][CPL];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if constexpr (CPL == 2) {
                const double2 t = *reinterpret_cast<const double2*>(xr + (size_t)q * ld);
                x[q][0] = t.x;
                x[q][1] = t.y;
            } else {
                x[q][0] = xr[(size_t)q * ld];
            }
        }
        const double* __restrict__ vb = v + (size_t)(b - b0) * (NI * 4);
#pragma unroll
        for (int a = 0; a < NI; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double m = vb[a * 4 + q];
#pragma unroll
                for (int c = 0; c < CPL; ++c) acc[a][c] = fma(m, x[q][c], acc[a][c]);
            }
    }
    // 1-orbital neighbours
    const double* __restrict__ vh = v + (size_t)(bs - b0) * (NI * 4);
#pragma unroll 4
    for (int b = bs; b < b1; ++b) {
        const int o = borb[b];
        const double* __restrict__ xr = Xg + (size_t)o * ld + c0;
        double x[CPL];
        if constexpr (CPL == 2) {
            const double2 t = *reinterpret_cast<const double2*>(xr);
            x[0] = t.x;
            x[1] = t.y;
        } else {
            x[0] = xr[0];
        }
        const double* __restrict__ vb = vh + (size_t)(b - bs) * NI;
#pragma unroll
        for (int a = 0; a < NI; ++a) {
            const double m = vb[a];
#pragma unroll
            for (int c = 0; c < CPL; ++c) acc[a][c] = fma(m, x[c], acc[a][c]);
        }
    }
}

template <int CPL>
__device__ __forceinline__ void load_cols(const double* p, size_t idx, double (&r)[CPL]) {
    if constexpr (CPL == 2) {
        const double2 t = *reinterpret_cast<const double2*>(p + idx);
        r[0] = t.x;
        r[1] = t.y;
    } else {
        r[0] = p[idx];
    }
}

template <int CPL>
__device__ __forceinline__ void store_cols(double* p, size_t idx, const double (&r)[CPL]) {
    if constexpr (CPL == 2) {
        *reinterpret_cast<double2*>(p + idx) = make_double2(r[0], r[1]);
    } else {
        p[idx] = r[0];
    }
}

template <int KIND, int NI, int CPL>
__device__ __forceinline__ void epilogue(const PassArgs& a, int row, int c0, const double (&acc)[NI][CPL], int arow,
                                         const double (&colA)[CPL], const double (&colB)[CPL],
                                         const int (&coln)[CPL], const int (&colr)[CPL], const double (&colal)[CPL],
                                         double (&d0)[CPL], double (&d1)[CPL]) {
    const size_t idx = (size_t)row * a.ld + c0;
    if constexpr (KIND == PASS_PLAIN) {
        double y[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) y[c] = acc[arow][c];
        store_cols<CPL>(a.Xio, idx, y);
    } else if constexpr (KIND == PASS_LANCZOS_A) {
        // colA = 1/beta_{n-1}, colB = beta_{n-1}/beta_{n-2}
        double tp[CPL], vq[CPL], sp[CPL], x1[CPL];
        load_cols<CPL>(a.S, idx, tp);
        load_cols<CPL>(a.Vq, idx, vq);
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            if (coln[c] == 0) {
                sp[c] = (row == colr[c]) ? 1.0 : 0.0;
            } else {
                sp[c] = acc[arow][c] * colA[c] - colB[c] * tp[c];
                d0[c] = fma(vq[c] * colA[c], sp[c], d0[c]);
            }
            x1[c] = a.g0 * sp[c];
        }
        store_cols<CPL>(a.S, idx, sp);
        store_cols<CPL>(a.Xio, idx, x1);
    } else {
        double xk[CPL], xp[CPL], s[CPL], xn[CPL];
        load_cols<CPL>(a.Xg, idx, xk);
        if (a.has_prev) {
            load_cols<CPL>(a.Xio, idx, xp);
        } else {
#pragma unroll
            for (int c = 0; c < CPL; ++c) xp[c] = 0.0;
        }
        load_cols<CPL>(a.S, idx, s);
#pragma unroll
        for (int c = 0; c < CPL; ++c) xn[c] = xk[c] + a.omega * (xk[c] - xp[c]) + a.gamma * (s[c] - acc[arow][c]);
        if constexpr (KIND == PASS_CHEB) {
            store_cols<CPL>(a.Xio, idx, xn);
        } else {
            double vq[CPL], tn[CPL];
            load_cols<CPL>(a.Vq, idx, vq);
            load_cols<CPL>(a.Tn, idx, tn);
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                if (coln[c] != 0) {
                    const double f = colal[c] * colA[c];
                    xn[c] -= f * vq[c];
                    s[c] -= f * tn[c];
                }
                d0[c] = fma(xn[c], s[c], d0[c]);
                d1[c] = fma(s[c], s[c], d1[c]);
            }
            store_cols<CPL>(a.Xio, idx, xn);
            store_cols<CPL>(a.S, idx, s);
        }
    }
}

template <int KIND, int CPL>
__global__ __launch_bounds__(kBlock) void pass_kernel(PassArgs a, const int* __restrict__ brow,
                                                      const int* __restrict__ bsplit, const int* __restrict__ borb,
                                                      const int64_t* __restrict__ voff,
                                                      const double* __restrict__ vals,
                                                      const int* __restrict__ atom_off) {
    // XCD-aware placement: workgroups are dispatched round-robin over the 8
    // XCDs (workgroup L runs on XCD L % 8).  XCD x owns the x-th eighth of the
    // slabs -- a compact region of space, since atoms are numbered with
    // spatial locality -- and walks it tile by tile, so the right-hand-side
    // rows its slabs gather (the region plus a cutoff halo) stay in its L2.
    const int s8 = a.n_slabs >> 3;
    const int L = blockIdx.x;
    const int k = L >> 3;
    const int tile = k / s8;
    const int slab = (L & 7) * s8 + (k - tile * s8);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c0 = tile * (kWave * CPL) + lane * CPL;

    double colA[CPL], colB[CPL], colal[CPL];
    int coln[CPL], colr[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        colA[c] = colB[c] = colal[c] = 0.0;
        coln[c] = 0;
        colr[c] = -1;
    }
    if constexpr (KIND == PASS_LANCZOS_A || KIND == PASS_CHEB_LAST) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            colA[c] = a.inv_beta[c0 + c];
            coln[c] = a.slot_n[c0 + c];
            colr[c] = a.slot_row[c0 + c];
            if constexpr (KIND == PASS_LANCZOS_A) colB[c] = a.coefT[c0 + c];
            if constexpr (KIND == PASS_CHEB_LAST) colal[c] = a.alpha[c0 + c];
        }
    }
    double d0[CPL], d1[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) d0[c] = d1[c] = 0.0;

    const int first = slab * a.atoms_per_slab;
    const int last = min(first + a.atoms_per_slab, a.n_atoms);  // empty for trailing slabs
    for (int I = first + wave; I < last; I += kWavesPerBlock) {
        if (atom_off[I + 1] - atom_off[I] == 4) {
            double acc[4][CPL];
            row_product<4, CPL>(I, a.ld, c0, a.Xg, brow, bsplit, borb, voff, vals, acc);
            const int r0 = atom_off[I];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                epilogue<KIND, 4, CPL>(a, r0 + q, c0, acc, q, colA, colB, coln, colr, colal, d0, d1);
        } else {
            double acc[1][CPL];
            row_product<1, CPL>(I, a.ld, c0, a.Xg, brow, bsplit, borb, voff, vals, acc);
            epilogue<KIND, 1, CPL>(a, atom_off[I], c0, acc, 0, colA, colB, coln, colr, colal, d0, d1);
        }
    }
    if constexpr (KIND == PASS_LANCZOS_A || KIND == PASS_CHEB_LAST) {
        __shared__ double red[2][kWavesPerBlock][kWave * CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            red[0][wave][lane * CPL + c] = d0[c];
            red[1][wave][lane * CPL + c] = d1[c];
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                double s0 = 0.0, s1 = 0.0;
#pragma unroll
                for (int w = 0; w < kWavesPerBlock; ++w) {
                    s0 += red[0][w][lane * CPL + c];
                    s1 += red[1][w][lane * CPL + c];
                }
                a.part0[(size_t)slab * a.ld + c0 + c] = s0;
                if constexpr (KIND == PASS_CHEB_LAST) a.part1[(size_t)slab * a.ld + c0 + c] = s1;
            }
        }
    }
}

template <int KIND>
static void launch_kind(const PassArgs& a, int cpl, hipStream_t st) {
    const int nwg = a.n_slabs * a.n_tiles;
    if (cpl == 2)
        hipLaunchKernelGGL((pass_kernel<KIND, 2>), dim3(nwg), dim3(kBlock), 0, st, a, a.brow, a.bsplit, a.borb,
                           a.voff, a.vals, a.atom_off);
    else
        hipLaunchKernelGGL((pass_kernel<KIND, 1>), dim3(nwg), dim3(kBlock), 0, st, a, a.brow, a.bsplit, a.borb,
                           a.voff, a.vals, a.atom_off);
}

void launch_pass(PassKind kind, const PassArgs& a, hipStream_t st) {
    const int cpl = a.ld / (a.n_tiles * kWave);
    switch (kind) {
        case PASS_LANCZOS_A: launch_kind<PASS_LANCZOS_A>(a, cpl, st); break;
        case PASS_CHEB: launch_kind<PASS_CHEB>(a, cpl, st); break;
        case PASS_CHEB_LAST: launch_kind<PASS_CHEB_LAST>(a, cpl, st); break;
        case PASS_PLAIN: launch_kind<PASS_PLAIN>(a, cpl, st); break;
    }
}

}  // namespace elses
