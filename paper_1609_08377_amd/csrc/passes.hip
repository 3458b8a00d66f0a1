// Fused sparse vector passes over the atom-block matrices (gfx950).
//
// Every pass multiplies one sparse matrix (A or B) with a block of right-hand
// sides stored [M][ld] (ld = slots, one right-hand side per lane), and fuses
// the element-wise work of one solver step into the epilogue, so the vectors
// cross HBM as few times as possible:
//
//   PASS_LANCZOS_A  w = A q_n; s' = w - beta_{n-1} t_{n-1}; partial q_n.s'
//                   (alpha_n).  Slots at n = 0 take s' = e_j instead (start
//                   vector B^{-1} e_j).
//   PASS_STEP_FIRST first Richardson step of the overlap solve B v = s with
//                   s = s' - alpha_n t_n: the operand x_1 = g0 s is formed
//                   from s' and t_n while gathering; s is stored for the
//                   later steps.
//   PASS_STEP       x_{k+1} = x_k + tau_k (s - B x_k)
//   PASS_STEP_LAST  the last step, v = x_d, with partial dots v.s and s.s
//                   (beta_n^2 and ||s||^2).
//   PASS_PLAIN      y = X x.
//
// Mixed precision (FP32 matrix values, FP32 overlap-solve vectors, FP64
// Lanczos vectors and scalars):
//   PASS_LANCZOS_A_MX  as PASS_LANCZOS_A with FP32 values and FP64
//                      accumulation.
//   PASS_STEP32_FIRST  as PASS_STEP_FIRST with an FP32 iterate; writes s in
//                      FP64 and FP32.
//   PASS_STEP32        FP32 Richardson step on FP32 vectors.
//   PASS_REFINE        r = s - B x with FP64 accumulation of the FP32
//                      first-round solution x; writes r and the first
//                      correction iterate g0 r in FP32.
//   PASS_STEP32_LAST   last FP32 correction step d, then v = x + d in FP64
//                      and the partial dots v.s, s.s.
//   PASS_PLAIN32       y = X x in FP32.
//
// The overlap solve always runs on s itself, so v = p(B) s for the fixed
// Richardson polynomial p and the Lanczos vectors q = p(B) t stay consistent
// to rounding at every step.
//
// Matrix values are identical for all lanes of a wave, so they are read
// through the scalar unit; each lane streams its own right-hand side(s).
//
// Three gather strategies for the right-hand-side rows of the coupled atoms:
//   direct  one atom per wave, rows read through L1/L2 (pass_kernel);
//   staged  a workgroup takes a cluster of consecutive atoms (one per wave),
//           copies the union of their coupled rows for its 64-column tile into
//           LDS once, and every wave reads its gathers from LDS
//           (pass_lds_kernel, FP64 kinds only);
//   grouped a row group (a 4-orbital atom and the 1-orbital atoms it couples
//           to most strongly) shares every gathered row of the union of its
//           coupled atoms (pass_group_kernel).
#include <type_traits>

#include "internal.h"

namespace elses {

// Arithmetic types of each pass kind: TV matrix values, TX gathered vector,
// TA accumulation.
template <int KIND>
struct KindTypes {
    using TV = double;
    using TX = double;
    using TA = double;
};
template <>
struct KindTypes<PASS_LANCZOS_A_MX> {
    using TV = float;
    using TX = double;
    using TA = double;
};
template <>
struct KindTypes<PASS_STEP32> {
    using TV = float;
    using TX = float;
    using TA = float;
};
template <>
struct KindTypes<PASS_REFINE> {
    using TV = float;
    using TX = float;
    using TA = double;
};
template <>
struct KindTypes<PASS_STEP32_LAST> {
    using TV = float;
    using TX = float;
    using TA = float;
};
template <>
struct KindTypes<PASS_PLAIN32> {
    using TV = float;
    using TX = float;
    using TA = float;
};
template <>
struct KindTypes<PASS_STEP32_FIRST> {
    using TV = float;
    using TX = double;
    using TA = float;
};

template <int KIND>
constexpr bool kVec32 = std::is_same_v<typename KindTypes<KIND>::TX, float>;
// Column tiling: kinds over FP32 vectors use n_tiles32 (up to four columns
// per lane), except the refinement pass, whose FP64 accumulators and LDS
// partials make the FP64 tiling (up to two columns per lane) faster.
template <int KIND>
constexpr bool kTiles32 = kVec32<KIND> && KIND != PASS_REFINE;
template <int KIND>
constexpr bool kHasDots = KIND == PASS_LANCZOS_A || KIND == PASS_STEP_LAST || KIND == PASS_LANCZOS_A_MX ||
                          KIND == PASS_STEP32_LAST;
template <int KIND>
constexpr bool kHasD1 = KIND == PASS_STEP_LAST || KIND == PASS_STEP32_LAST;
template <int KIND>
constexpr bool kFirst = KIND == PASS_STEP_FIRST || KIND == PASS_STEP32_FIRST;

__device__ __forceinline__ double fmac(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fmac(float a, float b, float c) { return fmaf(a, b, c); }

// CPL consecutive columns of one row: 8- or 16-byte vector accesses.
template <int CPL, typename T>
__device__ __forceinline__ void load_cols(const T* p, size_t idx, T (&r)[CPL]) {
    if constexpr (CPL == 1) {
        r[0] = p[idx];
    } else if constexpr (std::is_same_v<T, double> && CPL == 2) {
        const double2 t = *reinterpret_cast<const double2*>(p + idx);
        r[0] = t.x;
        r[1] = t.y;
    } else if constexpr (std::is_same_v<T, double> && CPL == 4) {
        const double2 t = *reinterpret_cast<const double2*>(p + idx);
        const double2 u = *reinterpret_cast<const double2*>(p + idx + 2);
        r[0] = t.x;
        r[1] = t.y;
        r[2] = u.x;
        r[3] = u.y;
    } else if constexpr (std::is_same_v<T, float> && CPL == 2) {
        const float2 t = *reinterpret_cast<const float2*>(p + idx);
        r[0] = t.x;
        r[1] = t.y;
    } else {
        static_assert(std::is_same_v<T, float> && CPL == 4, "unsupported column group");
        const float4 t = *reinterpret_cast<const float4*>(p + idx);
        r[0] = t.x;
        r[1] = t.y;
        r[2] = t.z;
        r[3] = t.w;
    }
}

template <int CPL, typename T>
__device__ __forceinline__ void store_cols(T* p, size_t idx, const T (&r)[CPL]) {
    if constexpr (CPL == 1) {
        p[idx] = r[0];
    } else if constexpr (std::is_same_v<T, double> && CPL == 2) {
        *reinterpret_cast<double2*>(p + idx) = make_double2(r[0], r[1]);
    } else if constexpr (std::is_same_v<T, double> && CPL == 4) {
        *reinterpret_cast<double2*>(p + idx) = make_double2(r[0], r[1]);
        *reinterpret_cast<double2*>(p + idx + 2) = make_double2(r[2], r[3]);
    } else if constexpr (std::is_same_v<T, float> && CPL == 2) {
        *reinterpret_cast<float2*>(p + idx) = make_float2(r[0], r[1]);
    } else {
        static_assert(std::is_same_v<T, float> && CPL == 4, "unsupported column group");
        *reinterpret_cast<float4*>(p + idx) = make_float4(r[0], r[1], r[2], r[3]);
    }
}

// Row product of atom I with the gathered operand.  `Src` maps the first
// orbital o of a coupled atom (as stored in `bidx`) to the CPL values of row
// o + q for this lane.
// acc[R][:] = sum over the coupled atoms b of (R x n_b block) * (rows of b).
// Coupled atoms [b0, bs) carry 4 orbitals, [bs, b1) one; idx[b] locates the
// first row of atom b for `src`; the blocks' values are contiguous from v
// (the R x 4 blocks, then the R x 1 blocks, row-major).  A wave takes every
// KS-th coupled atom starting at `sub`.  Gathers are issued in chunks (two
// 4-orbital atoms or eight 1-orbital atoms) before their FMAs, so several L2
// round trips overlap within one wave.
template <int R, int CPL, int KS, typename TA, typename TV, typename Src>
__device__ __forceinline__ void block_product(int b0, int bs, int b1, int sub, const int* __restrict__ idx,
                                              const TV* __restrict__ v, const Src& src, TA (&acc)[R][CPL]) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[r][c] = TA(0);
    constexpr int C4 = 2, C1 = 8;
    int b = b0 + sub;
    for (; b + (C4 - 1) * KS < bs; b += C4 * KS) {
        TA x[C4][4][CPL];
#pragma unroll
        for (int j = 0; j < C4; ++j) {
            const int o = idx[b + j * KS];
#pragma unroll
            for (int q = 0; q < 4; ++q) src.get(o + q, x[j][q]);
        }
#pragma unroll
        for (int j = 0; j < C4; ++j) {
            const TV* __restrict__ vb = v + (size_t)(b + j * KS - b0) * (R * 4);
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const TA m = static_cast<TA>(vb[r * 4 + q]);
#pragma unroll
                    for (int c = 0; c < CPL; ++c) acc[r][c] = fmac(m, x[j][q][c], acc[r][c]);
                }
        }
    }
    for (; b < bs; b += KS) {
        const int o = idx[b];
        TA x[4][CPL];
#pragma unroll
        for (int q = 0; q < 4; ++q) src.get(o + q, x[q]);
        const TV* __restrict__ vb = v + (size_t)(b - b0) * (R * 4);
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const TA m = static_cast<TA>(vb[r * 4 + q]);
#pragma unroll
                for (int c = 0; c < CPL; ++c) acc[r][c] = fmac(m, x[q][c], acc[r][c]);
            }
    }
    const TV* __restrict__ vh = v + (size_t)(bs - b0) * (R * 4);
    b = bs + sub;
    for (; b + (C1 - 1) * KS < b1; b += C1 * KS) {
        TA x[C1][CPL];
#pragma unroll
        for (int j = 0; j < C1; ++j) src.get(idx[b + j * KS], x[j]);
#pragma unroll
        for (int j = 0; j < C1; ++j) {
            const TV* __restrict__ vb = vh + (size_t)(b + j * KS - bs) * R;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const TA m = static_cast<TA>(vb[r]);
#pragma unroll
                for (int c = 0; c < CPL; ++c) acc[r][c] = fmac(m, x[j][c], acc[r][c]);
            }
        }
    }
    for (; b < b1; b += KS) {
        TA x[CPL];
        src.get(idx[b], x);
        const TV* __restrict__ vb = vh + (size_t)(b - bs) * R;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const TA m = static_cast<TA>(vb[r]);
#pragma unroll
            for (int c = 0; c < CPL; ++c) acc[r][c] = fmac(m, x[c], acc[r][c]);
        }
    }
}

template <int NI, int CPL, typename TA, typename TV, typename Src>
__device__ __forceinline__ void row_product(int I, const int* __restrict__ brow, const int* __restrict__ bsplit,
                                            const int* __restrict__ bidx, const int64_t* __restrict__ voff,
                                            const TV* __restrict__ vals, const Src& src, TA (&acc)[NI][CPL]) {
    block_product<NI, CPL, 1>(brow[I], bsplit[I], brow[I + 1], 0, bidx, vals + voff[I], src, acc);
}

// Rows of a [M][ld] block in memory type TX, delivered as TA.
template <int CPL, typename TX, typename TA>
struct GlobalSrc {
    const TX* __restrict__ X;
    int ld, c0;
    __device__ __forceinline__ void get(int row, TA (&r)[CPL]) const {
        if constexpr (std::is_same_v<TX, TA>) {
            load_cols<CPL>(X, (size_t)row * ld + c0, r);
        } else {
            TX t[CPL];
            load_cols<CPL>(X, (size_t)row * ld + c0, t);
#pragma unroll
            for (int c = 0; c < CPL; ++c) r[c] = static_cast<TA>(t[c]);
        }
    }
};

// The first overlap-solve operand x_1 = g0 (s' - f t_n), formed from two
// gathered FP64 rows (f = alpha_n / beta_{n-1} per column: t_n is stored
// unnormalised).
template <int CPL, typename TA>
struct FirstSrc {
    const double* __restrict__ Sp;
    const double* __restrict__ T;
    int ld, c0;
    double g0;
    double f[CPL];
    __device__ __forceinline__ void get(int row, TA (&r)[CPL]) const {
        double sp[CPL], t[CPL];
        load_cols<CPL>(Sp, (size_t)row * ld + c0, sp);
        load_cols<CPL>(T, (size_t)row * ld + c0, t);
#pragma unroll
        for (int c = 0; c < CPL; ++c) r[c] = static_cast<TA>(g0 * fma(-f[c], t[c], sp[c]));
    }
};

// LDS tile [rows][64] doubles, one column per lane
struct LdsSrc {
    const double* tile;
    int lane;
    __device__ __forceinline__ void get(int row, double (&r)[1]) const { r[0] = tile[row * kWave + lane]; }
};

template <int KIND>
__device__ __forceinline__ const typename KindTypes<KIND>::TX* gather_src(const PassArgs& a) {
    if constexpr (kVec32<KIND>)
        return a.Xg32;
    else
        return a.Xg;
}

struct ColState {
    double A, B, al;
    int n, r;
};

// Gather source of a pass kind.
template <int KIND, int CPL>
__device__ __forceinline__ auto make_src(const PassArgs& a, int c0, const ColState (&cs)[CPL]) {
    using TA = typename KindTypes<KIND>::TA;
    using TX = typename KindTypes<KIND>::TX;
    if constexpr (kFirst<KIND>) {
        FirstSrc<CPL, TA> src{a.S, a.Tn, a.ld, c0, a.g0, {}};
#pragma unroll
        for (int c = 0; c < CPL; ++c) src.f[c] = cs[c].al * cs[c].A;
        return src;
    } else {
        return GlobalSrc<CPL, TX, TA>{gather_src<KIND>(a), a.ld, c0};
    }
}

// Region membership of (row, columns c0 .. c0+CPL-1); all set without a mask.
template <int CPL>
__device__ __forceinline__ void row_mask(const PassArgs& a, int row, int c0, bool (&in)[CPL]) {
    if (a.mask) {
        const uint64_t w = a.mask[(size_t)row * a.mask_words + (c0 >> 6)];
#pragma unroll
        for (int c = 0; c < CPL; ++c) in[c] = (w >> ((c0 & 63) + c)) & 1ull;
    } else {
#pragma unroll
        for (int c = 0; c < CPL; ++c) in[c] = true;
    }
}

template <int CPL, typename T>
__device__ __forceinline__ void apply_mask(const bool (&in)[CPL], T (&v)[CPL]) {
#pragma unroll
    for (int c = 0; c < CPL; ++c) v[c] = in[c] ? v[c] : T(0);
}

template <int KIND, int NI, int CPL, typename TA>
__device__ __forceinline__ void epilogue(const PassArgs& a, int row, int c0, const TA (&acc)[NI][CPL], int arow,
                                         const ColState (&cs)[CPL], double (&d0)[CPL], double (&d1)[CPL]) {
    const size_t idx = (size_t)row * a.ld + c0;
    bool in[CPL];
    row_mask<CPL>(a, row, c0, in);
    if constexpr (KIND == PASS_PLAIN || KIND == PASS_PLAIN32) {
        TA y[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) y[c] = acc[arow][c];
        apply_mask<CPL>(in, y);
        if constexpr (KIND == PASS_PLAIN)
            store_cols<CPL>(a.Xio, idx, y);
        else
            store_cols<CPL>(a.Xio32, idx, y);
    } else if constexpr (KIND == PASS_LANCZOS_A || KIND == PASS_LANCZOS_A_MX) {
        // cs.A = 1/beta_{n-1}, cs.B = beta_{n-1}/beta_{n-2}
        double tp[CPL], vq[CPL], sp[CPL];
        load_cols<CPL>(a.S, idx, tp);
        load_cols<CPL>(a.Vq, idx, vq);
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            if (cs[c].n == 0) {
                sp[c] = (row == cs[c].r) ? 1.0 : 0.0;
            } else {
                sp[c] = in[c] ? acc[arow][c] * cs[c].A - cs[c].B * tp[c] : 0.0;
                d0[c] = fma(vq[c] * cs[c].A, sp[c], d0[c]);
            }
        }
        store_cols<CPL>(a.S, idx, sp);
    } else if constexpr (KIND == PASS_STEP_FIRST || KIND == PASS_STEP32_FIRST) {
        // s = s' - alpha_n t_n on the own rows, then the first step from x_1 = g0 s
        double sp[CPL], tn[CPL], sv[CPL];
        load_cols<CPL>(a.S, idx, sp);
        load_cols<CPL>(a.Tn, idx, tn);
#pragma unroll
        for (int c = 0; c < CPL; ++c) sv[c] = in[c] ? fma(-(cs[c].al * cs[c].A), tn[c], sp[c]) : 0.0;
        store_cols<CPL>(a.Sout, idx, sv);
        if constexpr (KIND == PASS_STEP_FIRST) {
            double xn[CPL];
#pragma unroll
            for (int c = 0; c < CPL; ++c) xn[c] = in[c] ? a.g0 * sv[c] + a.tau * (sv[c] - acc[arow][c]) : 0.0;
            store_cols<CPL>(a.Xio, idx, xn);
        } else {
            float s32[CPL], xn[CPL];
            const float tau = static_cast<float>(a.tau);
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                s32[c] = static_cast<float>(sv[c]);
                const float x1 = static_cast<float>(a.g0 * sv[c]);
                xn[c] = in[c] ? fmaf(tau, s32[c] - acc[arow][c], x1) : 0.0f;
            }
            store_cols<CPL>(a.R32o, idx, s32);
            store_cols<CPL>(a.Xio32, idx, xn);
        }
    } else if constexpr (KIND == PASS_STEP || KIND == PASS_STEP_LAST) {
        double xk[CPL], s[CPL], xn[CPL];
        load_cols<CPL>(a.Xg, idx, xk);
        load_cols<CPL>(a.S, idx, s);
#pragma unroll
        for (int c = 0; c < CPL; ++c) xn[c] = xk[c] + a.tau * (s[c] - acc[arow][c]);
        apply_mask<CPL>(in, xn);
        if constexpr (KIND == PASS_STEP) {
            store_cols<CPL>(a.Xio, idx, xn);
        } else {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                d0[c] = fma(xn[c], s[c], d0[c]);
                d1[c] = fma(s[c], s[c], d1[c]);
            }
            store_cols<CPL>(a.Xio, idx, xn);
        }
    } else if constexpr (KIND == PASS_RESID || KIND == PASS_PSTEP) {
        double sv[CPL], y[CPL];
        load_cols<CPL>(a.S, idx, sv);
#pragma unroll
        for (int c = 0; c < CPL; ++c) y[c] = KIND == PASS_RESID ? sv[c] - acc[arow][c] : sv[c] + a.tau * acc[arow][c];
        apply_mask<CPL>(in, y);
        store_cols<CPL>(a.Xio, idx, y);
    } else if constexpr (KIND == PASS_REFINE) {
        double s[CPL];
        float r32[CPL], x32[CPL];
        load_cols<CPL>(a.S, idx, s);
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const double r = in[c] ? s[c] - acc[arow][c] : 0.0;
            r32[c] = static_cast<float>(r);
            x32[c] = static_cast<float>(a.g0 * r);
        }
        store_cols<CPL>(a.R32o, idx, r32);
        store_cols<CPL>(a.Xio32, idx, x32);
    } else {
        static_assert(KIND == PASS_STEP32 || KIND == PASS_STEP32_LAST, "unknown pass kind");
        float xk[CPL], r[CPL], xn[CPL];
        load_cols<CPL>(a.Xg32, idx, xk);
        load_cols<CPL>(a.R32, idx, r);
        const float tau = static_cast<float>(a.tau);
#pragma unroll
        for (int c = 0; c < CPL; ++c) xn[c] = fmaf(tau, r[c] - acc[arow][c], xk[c]);
        apply_mask<CPL>(in, xn);
        if constexpr (KIND == PASS_STEP32) {
            store_cols<CPL>(a.Xio32, idx, xn);
        } else {
            float x1[CPL];
            double s[CPL], v[CPL];
            load_cols<CPL>(a.Xr1, idx, x1);
            load_cols<CPL>(a.S, idx, s);
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                v[c] = in[c] ? static_cast<double>(x1[c]) + static_cast<double>(xn[c]) : 0.0;
                d0[c] = fma(v[c], s[c], d0[c]);
                d1[c] = fma(s[c], s[c], d1[c]);
            }
            store_cols<CPL>(a.Xio, idx, v);
        }
    }
}

template <int KIND, int CPL>
__device__ __forceinline__ void load_colstate(const PassArgs& a, int c0, ColState (&cs)[CPL]) {
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        cs[c] = {0.0, 0.0, 0.0, 0, -1};
        if constexpr (KIND == PASS_LANCZOS_A || KIND == PASS_LANCZOS_A_MX || kFirst<KIND>) {
            cs[c].A = a.inv_beta[c0 + c];
            cs[c].n = a.slot_n[c0 + c];
            cs[c].r = a.slot_row[c0 + c];
            if constexpr (kFirst<KIND>)
                cs[c].al = a.alpha[c0 + c];
            else
                cs[c].B = a.coefT[c0 + c];
        }
    }
}

// Reduce the per-lane dot partials over the waves of the workgroup and store
// one partial per (group, column).
template <int KIND, int CPL, int NW>
__device__ __forceinline__ void store_partials(const PassArgs& a, int group, int c0, int wave, int lane,
                                               const double (&d0)[CPL], const double (&d1)[CPL], double* red) {
    if constexpr (kHasDots<KIND>) {
        __syncthreads();
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            red[(0 * NW + wave) * (kWave * CPL) + lane * CPL + c] = d0[c];
            red[(1 * NW + wave) * (kWave * CPL) + lane * CPL + c] = d1[c];
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                double s0 = 0.0, s1 = 0.0;
                for (int w = 0; w < NW; ++w) {
                    s0 += red[(0 * NW + w) * (kWave * CPL) + lane * CPL + c];
                    s1 += red[(1 * NW + w) * (kWave * CPL) + lane * CPL + c];
                }
                a.part0[(size_t)group * a.ld + c0 + c] = s0;
                if constexpr (kHasD1<KIND>) a.part1[(size_t)group * a.ld + c0 + c] = s1;
            }
        }
    }
}

// XCD-aware placement: workgroups are dispatched round-robin over the 8 XCDs
// (workgroup L runs on XCD L % 8).  XCD x owns the x-th eighth of the groups
// -- a compact region of space, since atoms are numbered with spatial
// locality -- and walks it tile by tile, so the right-hand-side rows its
// groups gather (the region plus a cutoff halo) stay in its L2.
// place = 1 keeps the XCD's eighth of the groups but walks it with the tile
// index fastest (a smaller region, all columns); place = 2 ignores the XCDs
// (tile-major over all groups).  place = 3 splits the columns instead of
// space: with n_tiles a multiple of 8, XCD x owns tiles x, x+8, ... over all
// groups, so every right-hand-side row is fetched into exactly one XCD's L2
// per tile (no halo duplication between XCDs); with n_tiles dividing 8, the
// 8 / n_tiles XCDs sharing a tile split the groups into contiguous parts.
__device__ __forceinline__ void xcd_place(int n_groups, int n_tiles, int place, int& tile, int& group) {
    const int s8 = n_groups >> 3;
    const int L = blockIdx.x;
    const int x = L & 7;
    const int k = L >> 3;
    if (place == 0) {
        tile = k / s8;
        group = x * s8 + (k - tile * s8);
    } else if (place == 1) {
        tile = k % n_tiles;
        group = x * s8 + k / n_tiles;
    } else if (place == 3) {
        if (n_tiles >= 8) {
            const int tl = k / n_groups;
            tile = x + 8 * tl;
            group = k - tl * n_groups;
        } else {
            const int parts = 8 / n_tiles;
            const int gp = n_groups / parts;
            tile = x % n_tiles;
            group = (x / n_tiles) * gp + k;
        }
    } else {
        tile = L / n_groups;
        group = L - tile * n_groups;
    }
}

template <int KIND>
__device__ __forceinline__ int kind_tiles(const PassArgs& a) {
    if constexpr (kTiles32<KIND>)
        return a.n_tiles32;
    else
        return a.n_tiles;
}

template <int KIND, int CPL>
__global__ __launch_bounds__(kBlock) void pass_kernel(PassArgs a, const int* __restrict__ brow,
                                                      const int* __restrict__ bsplit, const int* __restrict__ borb,
                                                      const int64_t* __restrict__ voff,
                                                      const typename KindTypes<KIND>::TV* __restrict__ vals,
                                                      const int* __restrict__ atom_off) {
    using TA = typename KindTypes<KIND>::TA;
    using TX = typename KindTypes<KIND>::TX;
    int tile, slab;
    xcd_place(a.n_slabs, kind_tiles<KIND>(a), a.place, tile, slab);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c0 = tile * (kWave * CPL) + lane * CPL;
    ColState cs[CPL];
    load_colstate<KIND, CPL>(a, c0, cs);
    double d0[CPL], d1[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) d0[c] = d1[c] = 0.0;
    const auto src = make_src<KIND, CPL>(a, c0, cs);
    const int first = slab * a.atoms_per_slab;
    const int last = min(first + a.atoms_per_slab, a.n_atoms);  // empty for trailing slabs
    for (int I = first + wave; I < last; I += kWavesPerBlock) {
        if (atom_off[I + 1] - atom_off[I] == 4) {
            TA acc[4][CPL];
            row_product<4, CPL>(I, brow, bsplit, borb, voff, vals, src, acc);
            const int r0 = atom_off[I];
#pragma unroll
            for (int q = 0; q < 4; ++q) epilogue<KIND, 4, CPL>(a, r0 + q, c0, acc, q, cs, d0, d1);
        } else {
            TA acc[1][CPL];
            row_product<1, CPL>(I, brow, bsplit, borb, voff, vals, src, acc);
            epilogue<KIND, 1, CPL>(a, atom_off[I], c0, acc, 0, cs, d0, d1);
        }
    }
    __shared__ double red[2 * kWavesPerBlock * kWave * CPL];
    store_partials<KIND, CPL, kWavesPerBlock>(a, slab, c0, wave, lane, d0, d1, red);
}

// Staged variant: NW waves, cluster = atoms [cl_atom[g], cl_atom[g+1]) (at
// most NW), union rows cl_urow[cl_uoff[g] .. cl_uoff[g+1]) (at most NU) staged
// in LDS; bloc[b] is the LDS row of block b's first coupled orbital.
template <int KIND, int NW, int NU>
__global__ __launch_bounds__(NW* kWave) void pass_lds_kernel(PassArgs a, const int* __restrict__ brow,
                                                            const int* __restrict__ bsplit,
                                                            const int* __restrict__ bloc,
                                                            const int64_t* __restrict__ voff,
                                                            const double* __restrict__ vals,
                                                            const int* __restrict__ atom_off) {
    __shared__ double tile_x[NU * kWave];
    int tile, g;
    xcd_place(a.n_slabs, a.n_tiles, a.place, tile, g);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c0 = tile * kWave + lane;
    ColState cs[1];
    load_colstate<KIND, 1>(a, c0, cs);
    double d0[1] = {0.0}, d1[1] = {0.0};
    int first = 0, last = 0;
    if (g < a.n_clusters) {
        first = a.cl_atom[g];
        last = a.cl_atom[g + 1];
        const int u0 = a.cl_uoff[g], nu = a.cl_uoff[g + 1] - u0;
        const int* __restrict__ ur = a.cl_urow + u0;
        // stage the union rows of this column tile (one 512-byte row per wave
        // step), issuing four row loads before their LDS stores
        const auto gsrc = make_src<KIND, 1>(a, c0, cs);
        int u = wave;
        for (; u + 3 * NW < nu; u += 4 * NW) {
            double t[4][1];
#pragma unroll
            for (int j = 0; j < 4; ++j) gsrc.get(ur[u + j * NW], t[j]);
#pragma unroll
            for (int j = 0; j < 4; ++j) tile_x[(u + j * NW) * kWave + lane] = t[j][0];
        }
        for (; u < nu; u += NW) {
            double t[1];
            gsrc.get(ur[u], t);
            tile_x[u * kWave + lane] = t[0];
        }
    }
    __syncthreads();
    const LdsSrc src{tile_x, lane};
    const int I = first + wave;
    if (I < last) {
        if (atom_off[I + 1] - atom_off[I] == 4) {
            double acc[4][1];
            row_product<4, 1>(I, brow, bsplit, bloc, voff, vals, src, acc);
            const int r0 = atom_off[I];
#pragma unroll
            for (int q = 0; q < 4; ++q) epilogue<KIND, 4, 1>(a, r0 + q, c0, acc, q, cs, d0, d1);
        } else {
            double acc[1][1];
            row_product<1, 1>(I, brow, bsplit, bloc, voff, vals, src, acc);
            epilogue<KIND, 1, 1>(a, atom_off[I], c0, acc, 0, cs, d0, d1);
        }
    }
    // reuse the staged tile as the reduction buffer
    store_partials<KIND, 1, NW>(a, g, c0, wave, lane, d0, d1, tile_x);
}

// Grouped variant: a row group's R rows share every gathered right-hand-side
// row of the union of their coupled atoms; the dense R x n_J value blocks are
// read through the scalar unit.  KS waves split the union of one group (wave
// `sub` takes every KS-th union atom), so each wave's chain of dependent
// gathers is KS times shorter; the partial rows are summed through LDS.
constexpr int kMaxGroupRows = 4 + kGroupH;

template <int R, int CPL, int KS, typename TA, typename TV, typename Src>
__device__ __forceinline__ void group_partial(int u0, int u4, int u1, int sub, const int* __restrict__ uorb,
                                              const TV* __restrict__ v, const Src& src, TA* pw, int lane) {
    TA acc[R][CPL];
    block_product<R, CPL, KS>(u0, u4, u1, sub, uorb, v, src, acc);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < CPL; ++c) pw[(r * kWave + lane) * CPL + c] = acc[r][c];
}

// Two waves per group (KS = 2): each wave keeps the rows it finishes in
// registers and hands the other wave's rows over through LDS, half of the
// group's partial rows (rows of parity p go to wave p, at slot row / 2).
// Exactly one workgroup barrier.  Taken at two or more columns per lane, where
// the halved LDS lets more waves run, and for FP64 values at one column per
// lane.  FP32-valued passes over 64-wide region tiles ran faster with the
// generic hand-over below (measured on one device, tiles of the 50000-atom
// box: step pass 316 against 357 us, mixed A pass 1134 against 1405 us),
// while FP64-valued ones ran slower (multiple-Arnoldi B pass 123 against
// 115 us).
constexpr int kHalfRows = kMaxGroupRows / 2;

template <int KIND, int R, int CPL, typename TA, typename TV, typename Src>
__device__ __forceinline__ void group_rows2(const PassArgs& a, int u0, int u4, int u1, int sub,
                                            const int* __restrict__ uorb, const TV* __restrict__ v,
                                            const Src& src, TA* pg, int lane, const int* __restrict__ rows,
                                            int c0, const ColState (&cs)[CPL], double (&d0)[CPL],
                                            double (&d1)[CPL]) {
    TA acc[R][CPL];
    block_product<R, CPL, 2>(u0, u4, u1, sub, uorb, v, src, acc);
    TA* mine = pg + (size_t)sub * kHalfRows * kWave * CPL;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if ((r & 1) != sub)
#pragma unroll
            for (int c = 0; c < CPL; ++c) mine[((r >> 1) * kWave + lane) * CPL + c] = acc[r][c];
    __syncthreads();
    const TA* other = pg + (size_t)(1 - sub) * kHalfRows * kWave * CPL;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if ((r & 1) == sub) {
            TA t[1][CPL];
#pragma unroll
            for (int c = 0; c < CPL; ++c) t[0][c] = acc[r][c] + other[((r >> 1) * kWave + lane) * CPL + c];
            epilogue<KIND, 1, CPL>(a, rows[r], c0, t, 0, cs, d0, d1);
        }
}

template <int KIND, int CPL, int KS>
__global__ __launch_bounds__(kBlock) void pass_group_kernel(PassArgs a, const int* __restrict__ gR,
                                                            const int* __restrict__ groff,
                                                            const int* __restrict__ grows,
                                                            const int* __restrict__ guoff,
                                                            const int* __restrict__ gu4,
                                                            const int* __restrict__ guorb,
                                                            const int64_t* __restrict__ gvoff,
                                                            const typename KindTypes<KIND>::TV* __restrict__ vals) {
    using TA = typename KindTypes<KIND>::TA;
    using TX = typename KindTypes<KIND>::TX;
    constexpr int GPW = kWavesPerBlock / KS;  // groups per workgroup
    constexpr bool kHand = KS == 2 && (CPL >= 2 || sizeof(typename KindTypes<KIND>::TV) == 8);
    constexpr size_t kPartBytes = sizeof(TA) * kWavesPerBlock * (kHand ? kHalfRows : kMaxGroupRows) * kWave * CPL;
    constexpr size_t kRedBytes = sizeof(double) * 2 * kWavesPerBlock * kWave * CPL;
    __shared__ __align__(16) unsigned char smem[kPartBytes > kRedBytes ? kPartBytes : kRedBytes];
    TA* part = reinterpret_cast<TA*>(smem);
    int tile, slab;
    xcd_place(a.n_slabs, kind_tiles<KIND>(a), a.place, tile, slab);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sub = wave % KS, gi = wave / KS;
    // c0: column of the vectors; sc: index of the per-slot state.  With
    // region tiles the vectors hold one tile per row and the slab names the
    // tile of its slot state.
    int c0 = tile * (kWave * CPL) + lane * CPL, sc = c0;
    if (a.slab_tile) {
        c0 = lane * CPL;
        sc = a.slab_tile[slab] * (kWave * CPL) + c0;
    }
    ColState cs[CPL];
    load_colstate<KIND, CPL>(a, sc, cs);
    double d0[CPL], d1[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) d0[c] = d1[c] = 0.0;
    const auto src = make_src<KIND, CPL>(a, c0, cs);
    const int g = a.slab_group ? a.slab_group[slab * GPW + gi] : slab * GPW + gi;
    // a region tile whose columns have all finished is skipped
    const bool tile_done = a.tile_live && a.tile_live[a.slab_tile[slab]] == 0;
    const bool live = (a.slab_group ? g >= 0 : g < a.n_grp) && !tile_done;
    int R = 0;
    if constexpr (kHand) {
        if (live) {
            R = gR[g];
            const int u0 = guoff[g], u4 = gu4[g], u1 = guoff[g + 1];
            const auto* __restrict__ v = vals + gvoff[g];
            const int* __restrict__ rows = grows + groff[g];
            TA* pg = part + (size_t)(gi * 2) * kHalfRows * kWave * CPL;
            switch (R) {
                case 1: group_rows2<KIND, 1, CPL>(a, u0, u4, u1, sub, guorb, v, src, pg, lane, rows, c0, cs, d0, d1); break;
                case 4: group_rows2<KIND, 4, CPL>(a, u0, u4, u1, sub, guorb, v, src, pg, lane, rows, c0, cs, d0, d1); break;
                case 5: group_rows2<KIND, 5, CPL>(a, u0, u4, u1, sub, guorb, v, src, pg, lane, rows, c0, cs, d0, d1); break;
                case 6: group_rows2<KIND, 6, CPL>(a, u0, u4, u1, sub, guorb, v, src, pg, lane, rows, c0, cs, d0, d1); break;
                case 7: group_rows2<KIND, 7, CPL>(a, u0, u4, u1, sub, guorb, v, src, pg, lane, rows, c0, cs, d0, d1); break;
                default: group_rows2<KIND, 8, CPL>(a, u0, u4, u1, sub, guorb, v, src, pg, lane, rows, c0, cs, d0, d1); break;
            }
        } else {
            __syncthreads();
        }
        store_partials<KIND, CPL, kWavesPerBlock>(a, slab, c0, wave, lane, d0, d1, reinterpret_cast<double*>(smem));
        return;
    }
    TA* pw = part + (size_t)wave * kMaxGroupRows * kWave * CPL;
    if (live) {
        R = gR[g];
        const int u0 = guoff[g], u4 = gu4[g], u1 = guoff[g + 1];
        const auto* __restrict__ v = vals + gvoff[g];
        switch (R) {
            case 1: group_partial<1, CPL, KS>(u0, u4, u1, sub, guorb, v, src, pw, lane); break;
            case 4: group_partial<4, CPL, KS>(u0, u4, u1, sub, guorb, v, src, pw, lane); break;
            case 5: group_partial<5, CPL, KS>(u0, u4, u1, sub, guorb, v, src, pw, lane); break;
            case 6: group_partial<6, CPL, KS>(u0, u4, u1, sub, guorb, v, src, pw, lane); break;
            case 7: group_partial<7, CPL, KS>(u0, u4, u1, sub, guorb, v, src, pw, lane); break;
            default: group_partial<8, CPL, KS>(u0, u4, u1, sub, guorb, v, src, pw, lane); break;
        }
    }
    __syncthreads();
    if (live) {
        // wave `sub` of the group finishes rows sub, sub + KS, ...
        const int* __restrict__ rows = grows + groff[g];
        const TA* pg = part + (size_t)(gi * KS) * kMaxGroupRows * kWave * CPL;
        for (int r = sub; r < R; r += KS) {
            TA acc[1][CPL];
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                TA t = TA(0);
#pragma unroll
                for (int s = 0; s < KS; ++s) t += pg[((size_t)s * kMaxGroupRows * kWave + r * kWave + lane) * CPL + c];
                acc[0][c] = t;
            }
            epilogue<KIND, 1, CPL>(a, rows[r], c0, acc, 0, cs, d0, d1);
        }
    }
    store_partials<KIND, CPL, kWavesPerBlock>(a, slab, c0, wave, lane, d0, d1, reinterpret_cast<double*>(smem));
}

template <int KIND>
static const typename KindTypes<KIND>::TV* kind_vals(const PassArgs& a) {
    if constexpr (std::is_same_v<typename KindTypes<KIND>::TV, float>)
        return a.vals32;
    else
        return a.vals;
}

template <int KIND, int CPL>
static void launch_cpl(const PassArgs& a, int nwg, hipStream_t st) {
    const auto* vals = kind_vals<KIND>(a);
    if (a.staged == 9) {
        if (a.group_split == 4)
            hipLaunchKernelGGL((pass_group_kernel<KIND, CPL, 4>), dim3(nwg), dim3(kBlock), 0, st, a, a.g_R, a.g_roff,
                               a.g_rows, a.g_uoff, a.g_u4, a.g_uorb, a.g_voff, vals);
        else if (a.group_split == 2)
            hipLaunchKernelGGL((pass_group_kernel<KIND, CPL, 2>), dim3(nwg), dim3(kBlock), 0, st, a, a.g_R, a.g_roff,
                               a.g_rows, a.g_uoff, a.g_u4, a.g_uorb, a.g_voff, vals);
        else
            hipLaunchKernelGGL((pass_group_kernel<KIND, CPL, 1>), dim3(nwg), dim3(kBlock), 0, st, a, a.g_R, a.g_roff,
                               a.g_rows, a.g_uoff, a.g_u4, a.g_uorb, a.g_voff, vals);
    } else {
        hipLaunchKernelGGL((pass_kernel<KIND, CPL>), dim3(nwg), dim3(kBlock), 0, st, a, a.brow, a.bsplit, a.borb,
                           a.voff, vals, a.atom_off);
    }
}

template <int KIND>
static void launch_kind(const PassArgs& a, hipStream_t st) {
    const int tiles = kTiles32<KIND> ? a.n_tiles32 : a.n_tiles;
    const int nwg = a.n_slabs * tiles;
    if constexpr (!std::is_same_v<typename KindTypes<KIND>::TV, float>) {
        if (a.staged == 1) {
            hipLaunchKernelGGL((pass_lds_kernel<KIND, kStageWaves[0], kStageRows[0]>), dim3(nwg),
                               dim3(kStageWaves[0] * kWave), 0, st, a, a.brow, a.bsplit, a.bloc, a.voff, a.vals,
                               a.atom_off);
            return;
        }
        if (a.staged == 2) {
            hipLaunchKernelGGL((pass_lds_kernel<KIND, kStageWaves[1], kStageRows[1]>), dim3(nwg),
                               dim3(kStageWaves[1] * kWave), 0, st, a, a.brow, a.bsplit, a.bloc, a.voff, a.vals,
                               a.atom_off);
            return;
        }
    }
    const int cpl = a.ld / (tiles * kWave);
    if constexpr (kTiles32<KIND>) {
        if (cpl == 4) return launch_cpl<KIND, 4>(a, nwg, st);
    }
    if (cpl == 2)
        launch_cpl<KIND, 2>(a, nwg, st);
    else
        launch_cpl<KIND, 1>(a, nwg, st);
}

void launch_pass(PassKind kind, const PassArgs& a, hipStream_t st) {
    switch (kind) {
        case PASS_LANCZOS_A: launch_kind<PASS_LANCZOS_A>(a, st); break;
        case PASS_STEP: launch_kind<PASS_STEP>(a, st); break;
        case PASS_STEP_LAST: launch_kind<PASS_STEP_LAST>(a, st); break;
        case PASS_PLAIN: launch_kind<PASS_PLAIN>(a, st); break;
        case PASS_LANCZOS_A_MX: launch_kind<PASS_LANCZOS_A_MX>(a, st); break;
        case PASS_STEP32: launch_kind<PASS_STEP32>(a, st); break;
        case PASS_REFINE: launch_kind<PASS_REFINE>(a, st); break;
        case PASS_STEP32_LAST: launch_kind<PASS_STEP32_LAST>(a, st); break;
        case PASS_PLAIN32: launch_kind<PASS_PLAIN32>(a, st); break;
        case PASS_STEP_FIRST: launch_kind<PASS_STEP_FIRST>(a, st); break;
        case PASS_STEP32_FIRST: launch_kind<PASS_STEP32_FIRST>(a, st); break;
        case PASS_RESID: launch_kind<PASS_RESID>(a, st); break;
        case PASS_PSTEP: launch_kind<PASS_PSTEP>(a, st); break;
    }
}

// Start of the overlap solve, element-wise over [M][vw]: s = s' - (alpha_n /
// beta_{n-1}) t_n (t_n stored unnormalised), x_1 = g0 s.  The slot of
// (row, c) is c, or with region tiles row_tile[row] * vw + c.  FP32 copies
// of s and x_1 are written when S32 is given.
__global__ void overlap_start_kernel(int64_t n, int vw, const double* __restrict__ Sp, const double* __restrict__ Tn,
                                     const double* __restrict__ alpha, const double* __restrict__ inv_beta,
                                     const int* __restrict__ row_tile, double g0, double* __restrict__ S,
                                     double* __restrict__ X1, float* __restrict__ S32, float* __restrict__ X132) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int row = (int)(e / vw), c = (int)(e - (int64_t)row * vw);
    const int slot = row_tile ? row_tile[row] * vw + c : c;
    const double sv = fma(-(alpha[slot] * inv_beta[slot]), Tn[e], Sp[e]);
    const double x1 = g0 * sv;
    if (S32) {
        S32[e] = static_cast<float>(sv);
        X132[e] = static_cast<float>(x1);
        S[e] = sv;
    } else {
        S[e] = sv;
        X1[e] = x1;
    }
}

void launch_overlap_start(int M, int vw, const double* Sp, const double* Tn, const double* alpha,
                          const double* inv_beta, const int* row_tile, double g0, double* S, double* X1, float* S32,
                          float* X132, hipStream_t st) {
    const int64_t n = (int64_t)M * vw;
    hipLaunchKernelGGL(overlap_start_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, vw, Sp, Tn,
                       alpha, inv_beta, row_tile, g0, S, X1, S32, X132);
}

// out[c] = sum_k part[k*ld + c] in two deterministic stages:
// stage 1 sums blocks of 64 partials per column, stage 2 the block sums.
__global__ void col_reduce1_kernel(const double* __restrict__ part, int n_part, int ld, double* __restrict__ tmp) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ld) return;
    const int k0 = blockIdx.y * 64, k1 = min(k0 + 64, n_part);
    double s = 0.0;
    for (int k = k0; k < k1; ++k) s += part[(size_t)k * ld + c];
    tmp[(size_t)blockIdx.y * ld + c] = s;
}

__global__ void col_reduce2_kernel(const double* __restrict__ tmp, int nb, int ld, const int* __restrict__ slot_n,
                                   const int* __restrict__ slot_row, double* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ld) return;
    double s = 0.0;
    for (int k = 0; k < nb; ++k) s += tmp[(size_t)k * ld + c];
    if (slot_n) s = (slot_n[c] == 0 || slot_row[c] < 0) ? 0.0 : s;
    out[c] = s;
}

__global__ void col_reduce_tiles1_kernel(const double* __restrict__ part, int L, const int* __restrict__ s0,
                                         const int* __restrict__ s1, double* __restrict__ tmp) {
    const int k = blockIdx.x;
    for (int c = threadIdx.x; c < L; c += blockDim.x) {
        double s = 0.0;
        for (int q = s0[k]; q < s1[k]; ++q) s += part[(size_t)q * L + c];
        tmp[(size_t)k * L + c] = s;
    }
}

__global__ void col_reduce_tiles2_kernel(const double* __restrict__ tmp, int L, int n_slots,
                                         const int* __restrict__ tile_chunk_off, const int* __restrict__ slot_n,
                                         const int* __restrict__ slot_row, double* __restrict__ out) {
    const int sidx = blockIdx.x * blockDim.x + threadIdx.x;
    if (sidx >= n_slots) return;
    const int t = sidx / L, c = sidx - t * L;
    double s = 0.0;
    for (int k = tile_chunk_off[t]; k < tile_chunk_off[t + 1]; ++k) s += tmp[(size_t)k * L + c];
    if (slot_n) s = (slot_n[sidx] == 0 || slot_row[sidx] < 0) ? 0.0 : s;
    out[sidx] = s;
}

void launch_col_reduce_tiles(const double* part, int L, int n_tiles, int n_chunks, const int* chunk_s0,
                             const int* chunk_s1, const int* tile_chunk_off, double* tmp, const int* slot_n,
                             const int* slot_row, double* out, hipStream_t st) {
    hipLaunchKernelGGL(col_reduce_tiles1_kernel, dim3(n_chunks), dim3(L), 0, st, part, L, chunk_s0, chunk_s1, tmp);
    const int n_slots = n_tiles * L;
    hipLaunchKernelGGL(col_reduce_tiles2_kernel, dim3((n_slots + 255) / 256), dim3(256), 0, st, tmp, L, n_slots,
                       tile_chunk_off, slot_n, slot_row, out);
}

void launch_col_reduce(const double* part, int n_part, int ld, double* tmp, const int* slot_n, const int* slot_row,
                       double* out, hipStream_t st) {
    const int nb = (n_part + 63) / 64;
    hipLaunchKernelGGL(col_reduce1_kernel, dim3((ld + 255) / 256, nb), dim3(256), 0, st, part, n_part, ld, tmp);
    hipLaunchKernelGGL(col_reduce2_kernel, dim3((ld + 255) / 256), dim3(256), 0, st, tmp, nb, ld, slot_n, slot_row,
                       out);
}

}  // namespace elses
