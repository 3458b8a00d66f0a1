// Region problems in a compact per-region layout, solved by one persistent
// launch (gfx950).
//
// The paper's real-space projection (Sec. III-B, III-C) solves each column's
// equations on the principal sub-pencil (A_r, B_r) of the atoms within a
// radius of the column's atom, one column per CPU core.  Here one workgroup
// owns one region at a time and runs its whole shifted solve (every outer
// Lanczos step, every overlap solve, the multi-shift update and the density
// assembly) without leaving the kernel; finished workgroups take the next
// region from a costliest-first device queue, so regions of uneven size and
// iteration count do not wait for each other (the load imbalance the paper
// measures as barrier time, Table II).  The host launches at most one
// workgroup per CU, and gives each region the Chebyshev-Richardson plan of
// its own overlap interval (degree, first step and roots per region).
//
// Layout of one region (built on the host, see build_compact):
//  - its m orbitals are permuted to positions 0..P-1 (P = 64 x slices), rows
//    sorted by their number of nonzeros, so that a slice of 64 consecutive
//    positions holds rows of nearly equal length; position p of a slice is
//    lane p % 64 of a wavefront;
//  - a slice stores its entries lane-interleaved (entry k of lane l at
//    k * 64 + l): a 16-bit column position and the values of A and B at that
//    entry (FP64, and FP32 for mixed precision), padded with zero values up
//    to the slice's longest row;
//  - every vector is [P][C] (C columns of the region side by side).
//
// Per workgroup, the iterate of the overlap solve lives in LDS (it is
// gathered by every sparse product of the inner iteration): in two buffers
// that the Richardson steps ping-pong between when both fit, else staged
// through the scratch area at each step; the Lanczos vectors live in a
// per-workgroup scratch area in global memory (touched a few times per
// outer step).
//
// The outer method is the same as in the global solver (shift.hip): a
// Lanczos process for B^{-1}A in the B inner product from B^{-1} e_j (Eqs.
// 13-14), the LU recurrences of (z_k I - T_n) for every shift, and the
// residual estimate |zeta/eta| ||s_n||.  All reductions are workgroup
// reductions in a fixed order.
#include <algorithm>

#include "internal.h"

namespace elses {

namespace {

constexpr int kRW = kRegThreads / 64;  // waves per workgroup

struct cplx {
    double r, i;
};
__device__ __forceinline__ cplx cmulx(cplx a, cplx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
// 1/a; |a| >= Im z > 0 and moderate here, so no scaling against overflow
__device__ __forceinline__ cplx cinvx(cplx a) {
    const double id = 1.0 / (a.r * a.r + a.i * a.i);
    return {a.r * id, -a.i * id};
}

// C consecutive values at p (aligned to C values)
template <int C, typename T>
__device__ __forceinline__ void ldv(const T* p, T (&v)[C]) {
    if constexpr (C == 4 && sizeof(T) == 4) {
        const float4 q = *reinterpret_cast<const float4*>(p);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else if constexpr (C == 2 && sizeof(T) == 4) {
        const float2 q = *reinterpret_cast<const float2*>(p);
        v[0] = q.x; v[1] = q.y;
    } else if constexpr (C == 4 && sizeof(T) == 8) {
        const double2 q0 = reinterpret_cast<const double2*>(p)[0];
        const double2 q1 = reinterpret_cast<const double2*>(p)[1];
        v[0] = q0.x; v[1] = q0.y; v[2] = q1.x; v[3] = q1.y;
    } else if constexpr (C == 2 && sizeof(T) == 8) {
        const double2 q = *reinterpret_cast<const double2*>(p);
        v[0] = q.x; v[1] = q.y;
    } else {
        v[0] = p[0];
    }
}
template <int C, typename T>
__device__ __forceinline__ void stv(T* p, const T (&v)[C]) {
    if constexpr (C == 4 && sizeof(T) == 4) {
        *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
    } else if constexpr (C == 2 && sizeof(T) == 4) {
        *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
    } else if constexpr (C == 4 && sizeof(T) == 8) {
        reinterpret_cast<double2*>(p)[0] = make_double2(v[0], v[1]);
        reinterpret_cast<double2*>(p)[1] = make_double2(v[2], v[3]);
    } else if constexpr (C == 2 && sizeof(T) == 8) {
        *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    } else {
        p[0] = v[0];
    }
}

// Sum of N values over the workgroup; every thread receives the sums.  Lanes
// are summed by a fixed butterfly, then the waves in order.
template <int N>
__device__ __forceinline__ void wg_sum(double (&v)[N], double* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < N; ++c)
        for (int o = 32; o > 0; o >>= 1) v[c] += __shfl_xor(v[c], o, 64);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < N; ++c) red[w * N + c] = v[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < N; ++c) {
        double t = 0.0;
        for (int q = 0; q < kRW; ++q) t += red[q * N + c];
        v[c] = t;
    }
    __syncthreads();
}

// acc = sum over the entries of one slice row (this lane's) of val * x[col],
// x gathered from src ([P][C] of type TX), accumulated in TA.  Entry k of
// the lane is at e0 + 64 k; offsets are 32-bit from uniform base pointers.
template <int C, typename TA, typename TV, typename TX>
__device__ __forceinline__ void row_product(const uint16_t* __restrict__ ib, const TV* __restrict__ vb, uint32_t e0,
                                            int len, const TX* src, TA (&acc)[C]) {
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = TA(0);
    const int main = len & ~15;
#pragma unroll 16
    for (int k = 0; k < main; ++k) {
        const uint32_t e = e0 + 64u * (uint32_t)k;
        const uint32_t j = ib[e];
        const TA v = static_cast<TA>(vb[e]);
        TX xv[C];
        ldv<C>(src + j * (uint32_t)C, xv);
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = fma(v, static_cast<TA>(xv[c]), acc[c]);
    }
    if (main < len) {
        // the last len - main (< 16) entries as one batch of loads; slots past
        // the end re-read the last entry (a cache hit) with weight zero
        uint32_t j[16];
        TV v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const uint32_t e = e0 + 64u * (uint32_t)min(main + q, len - 1);
            j[q] = ib[e];
            v[q] = vb[e];
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            TX xv[C];
            ldv<C>(src + j[q] * (uint32_t)C, xv);
            const TA w = (main + q < len) ? static_cast<TA>(v[q]) : TA(0);
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c] = fma(w, static_cast<TA>(xv[c]), acc[c]);
        }
    }
}

// One lane's half row of B (the entries its row stores of the pairs split
// between the two rows): acc += val * x[col] gathered from src ([P][C] FP32),
// and the transpose half Ys[col] += val * xs (xs = the row's own x scaled by
// 2^sh) in 32-bit fixed point: the terms are rounded to the nearest integer
// (|term| < 2^(30 - L) for a region whose positions take at most 2^L - 1
// transpose terms, so no sum overflows) and summed by LDS integer atomics,
// which makes the sums independent of the order the waves reach them.
// Entries go in batches of 16 written in issue order (index and value loads,
// gathers, FMAs, atomics): an atomic is an ordered memory operation that
// later loads may not pass, so interleaving them per entry would serialise
// the loads.  The last batch re-reads the row's last entry in its unused
// slots, with weight zero and no atomic.
template <int C>
__device__ __forceinline__ void half_row(const uint16_t* __restrict__ ib, const float* __restrict__ vb, uint32_t e0,
                                         int len, const float* src, const float (&xs)[C], int* Ys,
                                         float (&acc)[C]) {
    for (int k0 = 0; k0 < len; k0 += 16) {
        uint32_t j[16];
        float v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const uint32_t e = e0 + 64u * (uint32_t)min(k0 + q, len - 1);
            j[q] = ib[e];
            v[q] = vb[e];
        }
        float xv[16][C];
#pragma unroll
        for (int q = 0; q < 16; ++q) ldv<C>(src + j[q] * (uint32_t)C, xv[q]);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const float w = (k0 + q < len) ? v[q] : 0.0f;
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c] = fmaf(w, xv[q][c], acc[c]);
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if (k0 + q < len) {
#pragma unroll
                for (int c = 0; c < C; ++c) atomicAdd(Ys + j[q] * (uint32_t)C + c, (int)rintf(v[q] * xs[c]));
            }
        }
    }
}

// Largest of m over the wave, folded into *slot (non-negative floats order as
// their bit patterns).
__device__ __forceinline__ void wave_max_into(unsigned int* slot, float m) {
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(slot, __float_as_uint(m));
}

// Per-region view of the arguments
template <typename TV>
struct RView {
    int m, P, ns, ncol;
    const int* slen;          // [ns] longest row of each slice
    const int* sent;          // [ns] first entry of each slice (relative to the region)
    const uint16_t* idx;      // entries: column position
    const TV* Av;             // entries: values of A (precision of the passes)
    const TV* Bv;             // entries: values of B
    const double* A64;        // entries: FP64 values (refinement and audits)
    const double* B64;
    const TV* Mv;             // entries: values of the learned preconditioner M (or null)
    // the region's Richardson plan (per round): degree d, first step g0, inverse roots tau[0 .. d-2]
    int d;
    double g0;
    const double* tau;
    // half layout of B (FP32 Richardson steps when the launch sets it)
    const int* hslen;         // [ns] longest half row of each slice
    const int* hsent;         // [ns] first half entry of each slice (relative to the region)
    const uint16_t* hidx;
    const float* hval;
    const float* hdiag;       // [P] diagonal
    int heb;                  // |half values| < 2^(heb - L), 2^L > most transpose terms of a position
};

// Per-column scalars of the region being solved, in LDS (uniform values kept
// out of the register file).
struct ColState {
    double alpha[4], bprev[4], beta[4], snorm[4], invb[4];
    int alive[4], nend[4], jpos[4], col[4], notconv[4];
    int fallback;  // the region's preconditioned overlap solve failed once: plain iteration from then on
};

template <typename TV>
__device__ __forceinline__ const TV* pick(const double* d, const float* f) {
    if constexpr (sizeof(TV) == 8)
        return d;
    else
        return f;
}

// One Richardson round X <- p(B) rhs:  x_1 = g0 rhs,
// x_{k+1} = x_k + tau_k (rhs - B x_k), k = 1 .. d-1, with TV arithmetic.
// rhs [P][C] (global, this lane's positions only), X [P][C] in LDS.  With a
// second LDS buffer the steps ping-pong between the two; otherwise the new
// iterate of a lane's rows goes through the per-workgroup block Xn (global,
// this lane's positions only) until every gather of the old one is done.
// The same round in FP32 with B in the half layout: per step, pass 1 takes
// the step with each row's gathered half (into the second iterate buffer) and
// forms the transpose half (fixed point, into Ys after the two iterate
// buffers); pass 2 subtracts tau times the transpose half and clears Ys.  The
// fixed-point scale of step k is 2^sh with sh = 30 - heb - e, max |x_k| < 2^e
// (from the previous pass) and heb = the region's value exponent bound plus
// L, so that every term |B_pq x_p| 2^sh < 2^(30 - L).
template <int C>
__device__ __forceinline__ void richardson_half(const CompactArgs& a, const RView<float>& R, const float* rhs,
                                                float* X) {
    __shared__ unsigned int xmax[2];  // max |x_k| of the current and the next iterate
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const float g0 = static_cast<float>(R.g0);
    int* Ys = reinterpret_cast<int*>(X + 2 * a.lds_half);
    if (threadIdx.x < 2) xmax[threadIdx.x] = 0u;
    __syncthreads();
    float m = 0.f;
    for (int sl = w; sl < R.ns; sl += kRW) {
        const int pos = sl * 64 + lane;
        float r[C];
        ldv<C>(rhs + (size_t)pos * C, r);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            r[c] *= g0;
            m = fmaxf(m, fabsf(r[c]));
            Ys[(size_t)pos * C + c] = 0;
        }
        stv<C>(X + (size_t)pos * C, r);
    }
    wave_max_into(&xmax[1], m);
    __syncthreads();
    float* cur = X;
    float* nxt = X + a.lds_half;
    for (int k = 1; k < R.d; ++k) {
        const float tau = static_cast<float>(R.tau[k - 1]);
        int ex = 0;
        (void)frexpf(__uint_as_float(xmax[k & 1]), &ex);
        const int sh = 30 - R.heb - ex;
        if (threadIdx.x == 0) xmax[(k + 1) & 1] = 0u;  // read two barriers ago; refilled in pass 2
        for (int sl = w; sl < R.ns; sl += kRW) {
            const int pos = sl * 64 + lane;
            float xo[C], xs[C], acc[C], r[C];
            ldv<C>(cur + (size_t)pos * C, xo);
            ldv<C>(rhs + (size_t)pos * C, r);
            const float dg = R.hdiag[pos];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                xs[c] = ldexpf(xo[c], sh);
                acc[c] = dg * xo[c];
            }
            half_row<C>(R.hidx, R.hval, (uint32_t)(R.hsent[sl] + lane), R.hslen[sl], cur, xs, Ys, acc);
            // the step without the transpose half, which pass 2 subtracts
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c] = xo[c] + tau * (r[c] - acc[c]);
            stv<C>(nxt + (size_t)pos * C, acc);
        }
        __syncthreads();
        float mm = 0.f;
        for (int sl = w; sl < R.ns; sl += kRW) {
            const int pos = sl * 64 + lane;
            float g[C];
            ldv<C>(nxt + (size_t)pos * C, g);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int t = Ys[(size_t)pos * C + c];
                Ys[(size_t)pos * C + c] = 0;
                g[c] = fmaf(-tau, ldexpf(static_cast<float>(t), -sh), g[c]);
                mm = fmaxf(mm, fabsf(g[c]));
            }
            stv<C>(nxt + (size_t)pos * C, g);
        }
        wave_max_into(&xmax[(k + 1) & 1], mm);
        __syncthreads();
        float* t = cur;
        cur = nxt;
        nxt = t;
    }
    if (cur != X) {
        for (int sl = w; sl < R.ns; sl += kRW) {
            const int pos = sl * 64 + lane;
            float xn[C];
            ldv<C>(cur + (size_t)pos * C, xn);
            stv<C>(X + (size_t)pos * C, xn);
        }
        __syncthreads();
    }
}

// HALF: the kernel carries the half-layout path (FP32, 1 or 2 columns, not
// preconditioned: the only launches the host sets it for).  Kept out of every
// other kernel, whose product loops the compiler serialises under the extra
// register pressure of code they never run.
template <int C, typename TV, bool HALF>
__device__ __forceinline__ void richardson(const CompactArgs& a, const RView<TV>& R, const TV* rhs, TV* X, TV* Xn) {
    if constexpr (HALF) {
        if (a.half) {
            richardson_half<C>(a, R, rhs, X);
            return;
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const TV g0 = static_cast<TV>(R.g0);
    for (int sl = w; sl < R.ns; sl += kRW) {
        const int pos = sl * 64 + lane;
        TV r[C];
        ldv<C>(rhs + (size_t)pos * C, r);
#pragma unroll
        for (int c = 0; c < C; ++c) r[c] *= g0;
        stv<C>(X + (size_t)pos * C, r);
    }
    __syncthreads();
    if (a.lds_half > 0) {
        // two LDS buffers: step k gathers from one and writes the other, so one
        // barrier per step ends both the gathers and the writes
        TV* cur = X;
        TV* nxt = X + a.lds_half;
        for (int k = 1; k < R.d; ++k) {
            const TV tau = static_cast<TV>(R.tau[k - 1]);
            for (int sl = w; sl < R.ns; sl += kRW) {
                const int pos = sl * 64 + lane;
                TV acc[C], r[C], xo[C], xn[C];
                row_product<C>(R.idx, R.Bv, (uint32_t)(R.sent[sl] + lane), R.slen[sl], cur, acc);
                ldv<C>(rhs + (size_t)pos * C, r);
                ldv<C>(cur + (size_t)pos * C, xo);
#pragma unroll
                for (int c = 0; c < C; ++c) xn[c] = xo[c] + tau * (r[c] - acc[c]);
                stv<C>(nxt + (size_t)pos * C, xn);
            }
            __syncthreads();
            TV* t = cur;
            cur = nxt;
            nxt = t;
        }
        if (cur != X) {
            for (int sl = w; sl < R.ns; sl += kRW) {
                const int pos = sl * 64 + lane;
                TV xn[C];
                ldv<C>(cur + (size_t)pos * C, xn);
                stv<C>(X + (size_t)pos * C, xn);
            }
            __syncthreads();
        }
        return;
    }
    for (int k = 1; k < R.d; ++k) {
        const TV tau = static_cast<TV>(R.tau[k - 1]);
        for (int sl = w; sl < R.ns; sl += kRW) {
            const int pos = sl * 64 + lane;
            TV acc[C], r[C], xo[C], xn[C];
            row_product<C>(R.idx, R.Bv, (uint32_t)(R.sent[sl] + lane), R.slen[sl], X, acc);
            ldv<C>(rhs + (size_t)pos * C, r);
            ldv<C>(X + (size_t)pos * C, xo);
#pragma unroll
            for (int c = 0; c < C; ++c) xn[c] = xo[c] + tau * (r[c] - acc[c]);
            stv<C>(Xn + (size_t)pos * C, xn);
        }
        __syncthreads();
        for (int sl = w; sl < R.ns; sl += kRW) {
            const int pos = sl * 64 + lane;
            TV xn[C];
            ldv<C>(Xn + (size_t)pos * C, xn);
            stv<C>(X + (size_t)pos * C, xn);
        }
        __syncthreads();
    }
}

// Preconditioned conjugate gradients with the learned M for B x = rhs, per
// column (TV vectors, FP64 dot products), the overlap solve of the
// preconditioned path: x_0 = 0, r = rhs, z = M r, p = z; q = B p,
// a = (r.z)/(p.q), x += a p, r -= a q until ||r|| <= tol ||rhs||; then
// z = M r, b = (r.z)_new/(r.z)_old, p = z + b p.  The vector being gathered
// (p for B, r for M) is staged in X (LDS); the lane's own x, r, p, q, z live
// in per-workgroup scratch.  Returns 1 when a curvature p.Bp or r.Mr was not
// positive (M not positive definite on the Krylov space) or the steps ran
// out: the caller then takes the plain iteration (CG's judge and fallback);
// otherwise x is left in X.
template <int C, typename TV>
__device__ __forceinline__ int pcg_round(const CompactArgs& a, const RView<TV>& R, const TV* rhs, TV* X, TV* Xo,
                                         TV* Ro, TV* Po, TV* Qo, TV* Zo, double tol, double* red,
                                         unsigned long long* products) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double rr0[C], rz[C];
#pragma unroll
    for (int c = 0; c < C; ++c) rr0[c] = 0.0;
    for (int sl = w; sl < R.ns; sl += kRW) {
        const int pos = sl * 64 + lane;
        TV r[C], zero[C];
        ldv<C>(rhs + (size_t)pos * C, r);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            zero[c] = TV(0);
            rr0[c] = fma((double)r[c], (double)r[c], rr0[c]);
        }
        stv<C>(Ro + (size_t)pos * C, r);
        stv<C>(Xo + (size_t)pos * C, zero);
        stv<C>(X + (size_t)pos * C, r);
    }
    wg_sum<C>(rr0, red);
#pragma unroll
    for (int c = 0; c < C; ++c) rz[c] = 0.0;
    for (int sl = w; sl < R.ns; sl += kRW) {
        const int pos = sl * 64 + lane;
        TV z[C], r[C];
        row_product<C>(R.idx, R.Mv, (uint32_t)(R.sent[sl] + lane), R.slen[sl], X, z);
        ldv<C>(Ro + (size_t)pos * C, r);
#pragma unroll
        for (int c = 0; c < C; ++c) rz[c] = fma((double)r[c], (double)z[c], rz[c]);
        stv<C>(Po + (size_t)pos * C, z);
    }
    wg_sum<C>(rz, red);  // its barriers also end every gather of r
    bool active[C];
    int fail = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        active[c] = rr0[c] > 0.0;
        if (active[c] && !(rz[c] > 0.0)) fail = 1;
    }
    unsigned long long nprod = 1;
    if (!fail) {
        for (int sl = w; sl < R.ns; sl += kRW) {
            const int pos = sl * 64 + lane;
            TV pv[C];
            ldv<C>(Po + (size_t)pos * C, pv);
            stv<C>(X + (size_t)pos * C, pv);
        }
        __syncthreads();
        int k = 0;
        for (; k < a.inner_max; ++k) {
            double pq[C];
#pragma unroll
            for (int c = 0; c < C; ++c) pq[c] = 0.0;
            for (int sl = w; sl < R.ns; sl += kRW) {
                const int pos = sl * 64 + lane;
                TV q[C], pv[C];
                row_product<C>(R.idx, R.Bv, (uint32_t)(R.sent[sl] + lane), R.slen[sl], X, q);
                ldv<C>(X + (size_t)pos * C, pv);
#pragma unroll
                for (int c = 0; c < C; ++c) pq[c] = fma((double)pv[c], (double)q[c], pq[c]);
                stv<C>(Qo + (size_t)pos * C, q);
            }
            wg_sum<C>(pq, red);
            TV al[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (active[c] && !(pq[c] > 0.0)) fail = 1;
                al[c] = (active[c] && pq[c] > 0.0) ? static_cast<TV>(rz[c] / pq[c]) : TV(0);
            }
            ++nprod;
            if (fail) break;
            double rr[C];
#pragma unroll
            for (int c = 0; c < C; ++c) rr[c] = 0.0;
            for (int sl = w; sl < R.ns; sl += kRW) {
                const int pos = sl * 64 + lane;
                TV x[C], pv[C], q[C], r[C];
                ldv<C>(Xo + (size_t)pos * C, x);
                ldv<C>(X + (size_t)pos * C, pv);
                ldv<C>(Qo + (size_t)pos * C, q);
                ldv<C>(Ro + (size_t)pos * C, r);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    x[c] += al[c] * pv[c];
                    r[c] -= al[c] * q[c];
                    rr[c] = fma((double)r[c], (double)r[c], rr[c]);
                }
                stv<C>(Xo + (size_t)pos * C, x);
                stv<C>(Ro + (size_t)pos * C, r);
            }
            wg_sum<C>(rr, red);
            bool all = true;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (active[c] && rr[c] <= tol * tol * rr0[c]) active[c] = false;
                all = all && !active[c];
            }
            if (all) break;
            // z = M r on r staged in X
            for (int sl = w; sl < R.ns; sl += kRW) {
                const int pos = sl * 64 + lane;
                TV r[C];
                ldv<C>(Ro + (size_t)pos * C, r);
                stv<C>(X + (size_t)pos * C, r);
            }
            __syncthreads();
            double rzn[C];
#pragma unroll
            for (int c = 0; c < C; ++c) rzn[c] = 0.0;
            for (int sl = w; sl < R.ns; sl += kRW) {
                const int pos = sl * 64 + lane;
                TV z[C], r[C];
                row_product<C>(R.idx, R.Mv, (uint32_t)(R.sent[sl] + lane), R.slen[sl], X, z);
                ldv<C>(Ro + (size_t)pos * C, r);
#pragma unroll
                for (int c = 0; c < C; ++c) rzn[c] = fma((double)r[c], (double)z[c], rzn[c]);
                stv<C>(Zo + (size_t)pos * C, z);
            }
            wg_sum<C>(rzn, red);
            ++nprod;
            TV be[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (active[c] && !(rzn[c] > 0.0)) fail = 1;
                be[c] = (active[c] && rz[c] > 0.0) ? static_cast<TV>(rzn[c] / rz[c]) : TV(0);
                if (active[c]) rz[c] = rzn[c];
            }
            if (fail) break;
            // p = z + b p (frozen columns keep their p; their step length is 0)
            for (int sl = w; sl < R.ns; sl += kRW) {
                const int pos = sl * 64 + lane;
                TV z[C], pv[C];
                ldv<C>(Zo + (size_t)pos * C, z);
                ldv<C>(Po + (size_t)pos * C, pv);
#pragma unroll
                for (int c = 0; c < C; ++c) pv[c] = active[c] ? z[c] + be[c] * pv[c] : pv[c];
                stv<C>(Po + (size_t)pos * C, pv);
                stv<C>(X + (size_t)pos * C, pv);
            }
            __syncthreads();
        }
        if (k >= a.inner_max) fail = 1;
    }
    if (threadIdx.x == 0) atomicAdd(products, nprod);
    if (fail) {
        __syncthreads();
        return 1;
    }
    __syncthreads();  // every gather of X done
    for (int sl = w; sl < R.ns; sl += kRW) {
        const int pos = sl * 64 + lane;
        TV x[C];
        ldv<C>(Xo + (size_t)pos * C, x);
        stv<C>(X + (size_t)pos * C, x);
    }
    __syncthreads();
    return 0;
}

// Scratch blocks of the preconditioned overlap solve ([P][C] of TV each)
template <typename TV>
struct PcgScratch {
    TV *x, *r, *p, *q, *z;
};

// One round of the overlap solve: X <- (approximately) B^{-1} rhs to tol.
// Plain: the fixed Chebyshev-Richardson polynomial (degree for the round's
// tolerance).  Preconditioned (PC): CG with the learned M, falling back to the
// plain polynomial for the rest of the region once M fails.
template <int C, typename TV, int PC>
__device__ __forceinline__ void overlap_round(const CompactArgs& a, const RView<TV>& R, const TV* rhs, TV* X, TV* Xn,
                                              const PcgScratch<TV>& ps, double tol, double* red, ColState& cs) {
    if constexpr (PC) {
        if (!cs.fallback) {
            const int f = pcg_round<C, TV>(a, R, rhs, X, ps.x, ps.r, ps.p, ps.q, ps.z, tol, red, a.products);
            if (!f) return;
            if (threadIdx.x == 0) {
                cs.fallback = 1;
                atomicAdd(a.n_fallback, 1);
            }
            __syncthreads();
        }
    }
    richardson<C, TV, PC == 0 && sizeof(TV) == 4 && C <= 2>(a, R, rhs, X, Xn);
    if (threadIdx.x == 0) atomicAdd(a.products, (unsigned long long)(R.d - 1));
}

// v = p(B) s for the region's columns: S, V [P][C] FP64 (global); Rw scratch
// [P][C] of TV (global); X the LDS iterate.  FP64: one round to inner_tol.
// Mixed: two FP32 rounds (to sqrt(inner_tol)) with the FP64-accumulated
// residual s - B x between them (iterative refinement).
template <int C, typename TV, int PC>
__device__ __forceinline__ void overlap_solve(const CompactArgs& a, const RView<TV>& R, const double* S, double* V,
                                              TV* Rw, TV* Xn, TV* X, const PcgScratch<TV>& ps, double* red,
                                              ColState& cs) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if constexpr (sizeof(TV) == 8) {
        overlap_round<C, TV, PC>(a, R, S, X, Xn, ps, a.inner_tol, red, cs);
        for (int sl = w; sl < R.ns; sl += kRW) {
            const int pos = sl * 64 + lane;
            double v[C];
            ldv<C>(X + (size_t)pos * C, v);
            stv<C>(V + (size_t)pos * C, v);
        }
    } else {
        const double rtol = sqrt(a.inner_tol);
        // round 1 on fl32(s)
        for (int sl = w; sl < R.ns; sl += kRW) {
            const int pos = sl * 64 + lane;
            double s[C];
            float f[C];
            ldv<C>(S + (size_t)pos * C, s);
#pragma unroll
            for (int c = 0; c < C; ++c) f[c] = static_cast<float>(s[c]);
            stv<C>(Rw + (size_t)pos * C, f);
        }
        __syncthreads();  // X may still be read by the previous product
        overlap_round<C, TV, PC>(a, R, Rw, X, Xn, ps, rtol, red, cs);
        // refinement: r = s - B x with FP64 accumulation; V = x
        for (int sl = w; sl < R.ns; sl += kRW) {
            const int pos = sl * 64 + lane;
            double acc[C], s[C], xd[C];
            float xo[C], f[C];
            row_product<C>(R.idx, R.Bv, (uint32_t)(R.sent[sl] + lane), R.slen[sl], X, acc);
            ldv<C>(S + (size_t)pos * C, s);
            ldv<C>(X + (size_t)pos * C, xo);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                xd[c] = static_cast<double>(xo[c]);
                f[c] = static_cast<float>(s[c] - acc[c]);
            }
            stv<C>(V + (size_t)pos * C, xd);
            stv<C>(Rw + (size_t)pos * C, f);
        }
        if (threadIdx.x == 0) atomicAdd(a.products, 1ull);
        __syncthreads();  // every gather of round 1's x done before round 2 overwrites it
        overlap_round<C, TV, PC>(a, R, Rw, X, Xn, ps, rtol, red, cs);
        for (int sl = w; sl < R.ns; sl += kRW) {
            const int pos = sl * 64 + lane;
            double v[C];
            float d[C];
            ldv<C>(V + (size_t)pos * C, v);
            ldv<C>(X + (size_t)pos * C, d);
#pragma unroll
            for (int c = 0; c < C; ++c) v[c] += static_cast<double>(d[c]);
            stv<C>(V + (size_t)pos * C, v);
        }
    }
}

// FP64 true residual ||e_j - (z_k B - A) x_k||_2 of column c for every shift,
// x [K][P] complex in position order (global); values TV upcast to FP64 (the
// residual of the pencil the solve used).
template <int C, typename TV>
__device__ __forceinline__ void audit_column(const CompactArgs& a, const RView<TV>& R, int c, int jpos, const double* x,
                             double* out, double* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = 0; k < a.K; ++k) {
        const double zr = a.z[2 * k], zi = a.z[2 * k + 1];
        const double* xk = x + (size_t)k * R.P * 2;
        double part[1] = {0.0};
                for (int sl = w; sl < R.ns; sl += kRW) {
            const int pos = sl * 64 + lane;
            const int e0 = R.sent[sl] + lane;
            const int len = R.slen[sl];
            double bxr = 0, bxi = 0, axr = 0, axi = 0;
            for (int q = 0; q < len; ++q) {
                const int j = R.idx[e0 + q * 64];
                const double bv = static_cast<double>(R.Bv[e0 + q * 64]);
                const double av = static_cast<double>(R.Av[e0 + q * 64]);
                const double xr = xk[2 * (size_t)j], xi = xk[2 * (size_t)j + 1];
                bxr = fma(bv, xr, bxr);
                bxi = fma(bv, xi, bxi);
                axr = fma(av, xr, axr);
                axi = fma(av, xi, axi);
            }
            const double rr = (pos == jpos ? 1.0 : 0.0) - (zr * bxr - zi * bxi - axr);
            const double ri = -(zr * bxi + zi * bxr - axi);
            part[0] += rr * rr + ri * ri;
        }
        wg_sum<1>(part, red);
        if (threadIdx.x == 0) out[k] = sqrt(part[0]);
    }
    (void)c;
}


template <int C, typename TV, int PC>
__device__ __forceinline__ void solve_region(const CompactArgs& a, const RegionDesc& D, int ri, double* vbase, TV* X,
                                             double* red, ColState& cs) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int K = a.K;
    RView<TV> R;
    R.m = D.m;
    R.ns = D.nslice;
    R.P = D.nslice * 64;
    R.ncol = D.ncol;
    R.d = a.rdeg[ri];
    R.g0 = a.rg0[ri];
    R.tau = a.rtau + (size_t)ri * a.tau_stride;
    R.slen = a.slice_len + D.slice0;
    R.sent = a.slice_ent + D.slice0;
    R.idx = a.idx + D.ent0;
    R.A64 = a.A64 + D.ent0;
    R.B64 = a.B64 + D.ent0;
    R.Av = pick<TV>(a.A64, a.A32) + D.ent0;
    R.Bv = pick<TV>(a.B64, a.B32) + D.ent0;
    R.Mv = PC ? pick<TV>(a.M64, a.M32) + D.ent0 : nullptr;
    if (a.half) {
        R.hslen = a.hslice_len + D.slice0;
        R.hsent = a.hslice_ent + D.slice0;
        R.hidx = a.hidx + D.hent0;
        R.hval = a.hval + D.hent0;
        R.hdiag = a.hdiag + D.pos0;
        R.heb = D.heb;
    }
    const int P = R.P;
    const size_t vs = (size_t)P * C;
    double* Q = vbase;
    double* T0 = Q + vs;
    double* T1 = T0 + vs;
    double* S = T1 + vs;
    double* V = S + vs;
    TV* Rw = reinterpret_cast<TV*>(V + vs);
    TV* Xn = reinterpret_cast<TV*>(V + 2 * vs);
    PcgScratch<TV> ps;
    ps.x = reinterpret_cast<TV*>(V + 3 * vs);
    ps.r = reinterpret_cast<TV*>(V + 4 * vs);
    ps.p = reinterpret_cast<TV*>(V + 5 * vs);
    ps.q = reinterpret_cast<TV*>(V + 6 * vs);
    ps.z = reinterpret_cast<TV*>(V + 7 * vs);

    // In mixed precision q_n is kept in LDS too (over the two FP32 iterate
    // buffers of the ping-pong, free between an outer step's overlap solve and
    // the next A product, exactly [P][C] FP64).  The A product then gathers q_n
    // from LDS like the B products gather the iterate.  (Not in the FP64
    // kernels: there it serialised the 4-column kernel's loops.)
    constexpr bool kQ = sizeof(TV) == 4;
    const bool qlds = kQ && a.lds_half > 0;
    double* Ql = reinterpret_cast<double*>(X);

    if (tid == 0) cs.fallback = 0;
    if (tid < C) {
        const int cc = tid < D.ncol ? tid : 0;  // padded columns repeat the first one; no output
        cs.col[tid] = D.col0 + cc;
        cs.jpos[tid] = a.col_pos[D.col0 + cc];
    }
    __syncthreads();
    // start: s = e_j, t_0 = 0
        for (int sl = w; sl < R.ns; sl += kRW) {
        const int pos = sl * 64 + lane;
        double e[C], zero[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            e[c] = (pos == cs.jpos[c]) ? 1.0 : 0.0;
            zero[c] = 0.0;
        }
        stv<C>(S + (size_t)pos * C, e);
        stv<C>(T0 + (size_t)pos * C, zero);
    }
    __syncthreads();
    overlap_solve<C, TV, PC>(a, R, S, V, Rw, Xn, X, ps, red, cs);
    __syncthreads();
    // beta_0^2 = e_j^T B^{-1} e_j = v_0[j]
    if (tid < C) {
        const double v0 = V[(size_t)cs.jpos[tid] * C + tid];
        cs.bprev[tid] = sqrt(fmax(v0, 0.0));
        cs.alive[tid] = (v0 > 0.0) ? 1 : 0;
        cs.invb[tid] = (v0 > 0.0) ? 1.0 / sqrt(v0) : 0.0;
        cs.nend[tid] = 0;
    }
    __syncthreads();
    // q_1 = v_0 / beta_0, t_1 = e_j / beta_0
        for (int sl = w; sl < R.ns; sl += kRW) {
        const int pos = sl * 64 + lane;
        double v[C], s[C];
        ldv<C>(V + (size_t)pos * C, v);
        ldv<C>(S + (size_t)pos * C, s);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            v[c] *= cs.invb[c];
            s[c] *= cs.invb[c];
        }
        stv<C>(Q + (size_t)pos * C, v);
        stv<C>(T1 + (size_t)pos * C, s);
        if (qlds) stv<C>(Ql + (size_t)pos * C, v);
    }
    __syncthreads();

    for (int n = 1;; ++n) {
        // w = A q_n (FP64 accumulation), alpha_n = q_n . w
        {
            double al[C];
#pragma unroll
            for (int c = 0; c < C; ++c) al[c] = 0.0;
            auto a_rows = [&](const double* qs) {
                for (int sl = w; sl < R.ns; sl += kRW) {
                    const int pos = sl * 64 + lane;
                    double acc[C], q[C];
                    row_product<C>(R.idx, R.Av, (uint32_t)(R.sent[sl] + lane), R.slen[sl], qs, acc);
                    ldv<C>(qs + (size_t)pos * C, q);
#pragma unroll
                    for (int c = 0; c < C; ++c) al[c] = fma(q[c], acc[c], al[c]);
                    stv<C>(S + (size_t)pos * C, acc);
                }
            };
            if constexpr (kQ) {
                if (qlds)
                    a_rows(Ql);
                else
                    a_rows(Q);
            } else {
                a_rows(Q);
            }
            wg_sum<C>(al, red);
            if (tid < C) cs.alpha[tid] = al[tid];
            if (tid == 0) atomicAdd(a.products, 1ull);
        }
        __syncthreads();
        // s = w - alpha_n t_n - beta_{n-1} t_{n-1}
                for (int sl = w; sl < R.ns; sl += kRW) {
            const int pos = sl * 64 + lane;
            double s[C], t1[C], t0[C];
            ldv<C>(S + (size_t)pos * C, s);
            ldv<C>(T1 + (size_t)pos * C, t1);
            ldv<C>(T0 + (size_t)pos * C, t0);
#pragma unroll
            for (int c = 0; c < C; ++c) s[c] = s[c] - cs.alpha[c] * t1[c] - cs.bprev[c] * t0[c];
            stv<C>(S + (size_t)pos * C, s);
        }
        // v = p(B) s
        overlap_solve<C, TV, PC>(a, R, S, V, Rw, Xn, X, ps, red, cs);
        // beta_n^2 = v . s and ||s||^2
        {
            double dots[2 * C];
#pragma unroll
            for (int c = 0; c < 2 * C; ++c) dots[c] = 0.0;
                        for (int sl = w; sl < R.ns; sl += kRW) {
                const int pos = sl * 64 + lane;
                double v[C], s[C];
                ldv<C>(V + (size_t)pos * C, v);
                ldv<C>(S + (size_t)pos * C, s);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    dots[c] = fma(v[c], s[c], dots[c]);
                    dots[C + c] = fma(s[c], s[c], dots[C + c]);
                }
            }
            wg_sum<2 * C>(dots, red);
            if (tid < C) {
                cs.beta[tid] = dots[tid];  // beta_n^2 for now
                cs.snorm[tid] = sqrt(fmax(dots[C + tid], 0.0));
                cs.notconv[tid] = 0;
            }
        }
        __syncthreads();
        // multi-shift recurrences: pivots, coefficients, residual estimates
        for (int p = tid; p < C * K; p += kRegThreads) {
            const int c = p / K, k = p - c * K;
            if (!cs.alive[c] || c >= D.ncol) continue;
            const size_t sk = (size_t)(D.col0 + c) * K + k;
            double* fac = a.fac + sk * 4;
            if (a.conv[sk] != 0) {
                fac[0] = fac[1] = fac[2] = fac[3] = 0.0;
                continue;
            }
            const double al = cs.alpha[c];
            const double bp = cs.bprev[c];
            const cplx z = {a.z[2 * k], a.z[2 * k + 1]};
            cplx eta, zeta;
            if (n == 1) {
                eta = {z.r - al, z.i};
                zeta = {bp, 0.0};
            } else {
                const cplx ieo = cinvx({a.eta[2 * sk], a.eta[2 * sk + 1]});
                const cplx zo = {a.zeta[2 * sk], a.zeta[2 * sk + 1]};
                zeta = cmulx(zo, {bp * ieo.r, bp * ieo.i});
                eta = {z.r - al - bp * bp * ieo.r, z.i - bp * bp * ieo.i};
            }
            const cplx ie = cinvx(eta);
            a.eta[2 * sk] = eta.r;
            a.eta[2 * sk + 1] = eta.i;
            a.zeta[2 * sk] = zeta.r;
            a.zeta[2 * sk + 1] = zeta.i;
            const cplx ratio = cmulx(zeta, ie);
            const double res = sqrt(ratio.r * ratio.r + ratio.i * ratio.i) * cs.snorm[c];
            a.res[sk] = res;
            fac[0] = ie.r;
            fac[1] = ie.i;
            fac[2] = zeta.r;
            fac[3] = zeta.i;
            if (res <= a.tol)
                a.conv[sk] = n;
            else
                atomicAdd(&cs.notconv[c], 1);
        }
        __syncthreads();
        // x and p on the carried rows (the column's pattern, or all positions)
        for (int c = 0; c < D.ncol; ++c) {
            if (!cs.alive[c]) continue;
            const int cl = D.col0 + c;
            const int full = a.carry_full[cl];
            const int len = full ? P : (int)(a.pat_off[cl + 1] - a.pat_off[cl]);
            const int* pp = a.pat_pos + a.pat_off[cl];
            double* xs = a.xs + (size_t)a.carry_off[cl] * 2;
            double* ps = a.ps + (size_t)a.carry_off[cl] * 2;
            const double* facc = a.fac + (size_t)cl * K * 4;
            const double bp = cs.bprev[c];
            const int tot = K * len;
            for (int idx = tid; idx < tot; idx += kRegThreads) {
                const int k = idx / len;
                const int e = idx - k * len;
                const double* f = facc + 4 * k;
                const double ier = f[0], iei = f[1];
                if (ier == 0.0 && iei == 0.0) continue;  // converged shift: frozen
                const int pos = full ? e : pp[e];
                const double q = pos >= 0 ? Q[(size_t)pos * C + c] : 0.0;
                const size_t o = 2 * (size_t)idx;
                double ur = q, ui = 0.0;
                if (n > 1) {
                    ur += bp * ps[o];
                    ui = bp * ps[o + 1];
                }
                const double pr = ur * ier - ui * iei, pi = ur * iei + ui * ier;
                ps[o] = pr;
                ps[o + 1] = pi;
                double xr = n > 1 ? xs[o] : 0.0, xi = n > 1 ? xs[o + 1] : 0.0;
                xr += f[2] * pr - f[3] * pi;
                xi += f[2] * pi + f[3] * pr;
                xs[o] = xr;
                xs[o + 1] = xi;
            }
        }
        __syncthreads();  // the update has read q_n and the counts are final
        // column ends: every shift converged, Krylov space exhausted (beta_n at
        // the rounding level), or max_outer
        if (tid < C) {
            const int c = tid;
            cs.invb[c] = 0.0;
            if (cs.alive[c]) {
                const double b2 = cs.beta[c];
                const double beta = sqrt(fmax(b2, 0.0));
                const bool breakdown = !(b2 > 0.0) || !(beta > 1e-13 * (fabs(cs.alpha[c]) + cs.bprev[c]));
                const bool done = (c < D.ncol) ? (cs.notconv[c] == 0) : true;
                if (done || breakdown || n >= a.max_outer) {
                    cs.alive[c] = 0;
                    cs.nend[c] = n;
                    if (c < D.ncol && cs.notconv[c] != 0) atomicAdd(a.n_notconv, 1);
                } else {
                    cs.invb[c] = 1.0 / beta;
                    cs.bprev[c] = beta;
                }
            }
        }
        __syncthreads();
        int any_alive = 0;
#pragma unroll
        for (int c = 0; c < C; ++c) any_alive |= cs.alive[c];
        if (!any_alive) break;
        // q_{n+1} = v / beta_n, t_{n-1} <- t_n, t_{n+1} = s / beta_n
                for (int sl = w; sl < R.ns; sl += kRW) {
            const int pos = sl * 64 + lane;
            double v[C], s[C], t1[C];
            ldv<C>(V + (size_t)pos * C, v);
            ldv<C>(S + (size_t)pos * C, s);
            ldv<C>(T1 + (size_t)pos * C, t1);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const double ib = cs.invb[c];
                v[c] *= ib;
                s[c] *= ib;
                t1[c] = ib != 0.0 ? t1[c] : 0.0;
            }
            stv<C>(Q + (size_t)pos * C, v);
            stv<C>(T0 + (size_t)pos * C, t1);
            stv<C>(T1 + (size_t)pos * C, s);
            if (qlds) stv<C>(Ql + (size_t)pos * C, v);
        }
        __syncthreads();
    }

    // outputs of the region's columns
    for (int c = 0; c < D.ncol; ++c) {
        const int cl = D.col0 + c;
        const int full = a.carry_full[cl];
        const int64_t p0 = a.pat_off[cl];
        const int plen = (int)(a.pat_off[cl + 1] - p0);
        const int clen = full ? P : plen;
        const int* pp = a.pat_pos + p0;
        const double* xs = a.xs + (size_t)a.carry_off[cl] * 2;
        if (a.x_out && !a.full_out) {
            double* dst = a.x_out + (size_t)p0 * K * 2;
            for (int idx = tid; idx < K * plen; idx += kRegThreads) {
                const int k = idx / plen;
                const int e = idx - k * plen;
                double vr = 0.0, vi = 0.0;
                if (!full) {
                    vr = xs[2 * (size_t)idx];
                    vi = xs[2 * (size_t)idx + 1];
                } else if (pp[e] >= 0) {
                    const size_t o = 2 * ((size_t)k * clen + pp[e]);
                    vr = xs[o];
                    vi = xs[o + 1];
                }
                dst[2 * (size_t)idx] = vr;
                dst[2 * (size_t)idx + 1] = vi;
            }
        }
        if (a.x_out && a.full_out) {
            // region vectors in the region's own orbital order
            double* dst = a.x_out + (size_t)a.full_off[cl] * K * 2;
            const uint16_t* prow = a.pos_row + D.pos0;
            for (int idx = tid; idx < K * P; idx += kRegThreads) {
                const int k = idx / P;
                const int pos = idx - k * P;
                const int row = prow[pos];
                if (row >= R.m) continue;
                const size_t o = 2 * ((size_t)k * R.m + row);
                dst[o] = xs[2 * (size_t)idx];
                dst[o + 1] = xs[2 * (size_t)idx + 1];
            }
        }
        if (a.rho_out || a.ctr_out) {
            double tr[2] = {0.0, 0.0};
            for (int e = tid; e < plen; e += kRegThreads) {
                const int src = full ? pp[e] : e;
                double r = 0.0;
                if (src >= 0)
                    for (int k = 0; k < K; ++k) {
                        const size_t o = 2 * ((size_t)k * clen + src);
                        r += a.cw[2 * k] * xs[o + 1] + a.cw[2 * k + 1] * xs[o];
                    }
                if (a.rho_out) a.rho_out[p0 + e] = r;
                tr[0] = fma(r, a.pat_B[p0 + e], tr[0]);
                tr[1] = fma(r, a.pat_A[p0 + e], tr[1]);
            }
            wg_sum<2>(tr, red);
            if (tid == 0 && a.ctr_out) {
                a.ctr_out[2 * (size_t)cl] = tr[0];
                a.ctr_out[2 * (size_t)cl + 1] = tr[1];
            }
        }
        if (a.iters_out && tid == 0) a.iters_out[cl] = cs.nend[c];
        if (a.resid_out) {
            if (full && a.audit) {
                audit_column<C, TV>(a, R, c, cs.jpos[c], xs, a.resid_out + (size_t)cl * K, red);
            } else {
                for (int k = tid; k < K; k += kRegThreads)
                    a.resid_out[(size_t)cl * K + k] = a.res[(size_t)cl * K + k];
            }
        }
    }
    __syncthreads();
}

template <typename TV, int C, int PC>
__global__ __launch_bounds__(kRegThreads, 2) void compact_kernel(CompactArgs a) {
    __shared__ double red[kRW * 8];
    __shared__ ColState cs;
    __shared__ int s_r;
    extern __shared__ __align__(16) unsigned char s_dyn[];
    TV* X = reinterpret_cast<TV*>(s_dyn);
    double* vbase = a.vec + (size_t)blockIdx.x * a.vec_stride;
    if (a.wg_clock && threadIdx.x == 0) a.wg_clock[2 * blockIdx.x] = wall_clock64();
    for (;;) {
        if (threadIdx.x == 0) s_r = atomicAdd(a.queue, 1);
        __syncthreads();
        const int r = s_r;
        __syncthreads();
        if (r >= a.n_regions) {
            if (a.wg_clock && threadIdx.x == 0) a.wg_clock[2 * blockIdx.x + 1] = wall_clock64();
            return;
        }
        const int ri = a.order[r];
        const RegionDesc D = a.reg[ri];
        solve_region<C, TV, PC>(a, D, ri, vbase, X, red, cs);
    }
}

template <typename TV, int PC>
const void* pick_kernel(int cw) {
    if (cw == 1) return reinterpret_cast<const void*>(&compact_kernel<TV, 1, PC>);
    if (cw == 2) return reinterpret_cast<const void*>(&compact_kernel<TV, 2, PC>);
    return reinterpret_cast<const void*>(&compact_kernel<TV, 4, PC>);
}

const void* kernel_for(bool fp64, int cw, bool pc) {
    if (pc) return fp64 ? pick_kernel<double, 1>(cw) : pick_kernel<float, 1>(cw);
    return fp64 ? pick_kernel<double, 0>(cw) : pick_kernel<float, 0>(cw);
}

__global__ void zero_ints_kernel(int* __restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

}  // namespace

void launch_zero_ints(int* p, size_t n, hipStream_t st) {
    const unsigned blocks = (unsigned)std::min<size_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(zero_ints_kernel, dim3(std::max(1u, blocks)), dim3(256), 0, st, p, n);
}

int compact_occupancy(bool fp64, int cw, bool precond, size_t lds) {
    const void* k = kernel_for(fp64, cw, precond);
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kRegThreads, lds) != hipSuccess) return 0;
    return nb;
}

void launch_compact(const CompactArgs& a, bool fp64, int cw, bool precond, int n_wg, size_t lds, hipStream_t st) {
    void* args[] = {const_cast<CompactArgs*>(&a)};
    (void)hipLaunchKernel(kernel_for(fp64, cw, precond), dim3(n_wg), dim3(kRegThreads), args, lds, st);
}

}  // namespace elses
