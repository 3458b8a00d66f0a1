// Learned block sparse approximate inverse of the overlap (gfx950 kernels).
//
// A small multilayer perceptron maps features of an atom pair (I, J) of B's
// block pattern to the block M_IJ of an approximate inverse M ~ B^{-1}; the
// preconditioned overlap solve then iterates x_{k+1} = x_k + tau_k M (s - B x_k).
//
// Features of a pair (I <= J), F = 40: displacement r_J - r_I / 4 A (3), its
// length / 4 A, 4-orbital flags of I and J, 10 B_IJ (4 x 4 zero-padded),
// 10 (E^2)_IJ with E = B - I (4 x 4), 1 if I == J, 0.
// Network: 40 -> 128 -> 128 -> 128 -> 16 with the exact GELU x Phi(x) after
// the hidden layers; parameters flat FP32: W1[128][40] b1 W2[128][128] b2
// W3[128][128] b3 W4[16][128] b4.
#include <math.h>

#include "internal.h"

namespace elses {

// ---------------------------------------------------------------------------
// Features, targets
// ---------------------------------------------------------------------------

__device__ __forceinline__ int find_block(const int* __restrict__ bcol, int b0, int b1, int J) {
    while (b0 < b1) {
        const int m = (b0 + b1) >> 1;
        if (bcol[m] < J)
            b0 = m + 1;
        else
            b1 = m;
    }
    return b0;
}

__global__ void spai_features_kernel(int64_t n, const int* __restrict__ pI, const int* __restrict__ pJ,
                                     const int* __restrict__ pb, const int* __restrict__ atom_off,
                                     const int* __restrict__ brow, const int* __restrict__ bcol,
                                     const int64_t* __restrict__ asc_voff, const double* __restrict__ Bv,
                                     const double* __restrict__ pos, double box, float* __restrict__ feat) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int I = pI[p], J = pJ[p];
    const int nI = atom_off[I + 1] - atom_off[I], nJ = atom_off[J + 1] - atom_off[J];
    float* f = feat + p * 40;
    double d[3];
    double r2 = 0.0;
    for (int c = 0; c < 3; ++c) {
        double t = pos[3 * J + c] - pos[3 * I + c];
        if (box > 0.0) t -= box * nearbyint(t / box);
        d[c] = t;
        r2 += t * t;
    }
    for (int c = 0; c < 3; ++c) f[c] = (float)(d[c] / 4.0);
    f[3] = (float)(sqrt(r2) / 4.0);
    f[4] = nI == 4 ? 1.f : 0.f;
    f[5] = nJ == 4 ? 1.f : 0.f;
    const double* bij = Bv + asc_voff[pb[p]];
    for (int e = 0; e < 16; ++e) {
        const int a = e >> 2, c = e & 3;
        f[6 + e] = (a < nI && c < nJ) ? (float)(10.0 * bij[a * nJ + c]) : 0.f;
    }
    // (E^2)_IJ = sum_K E_IK E_KJ over the atoms K coupled to I (and to J)
    double e2[4][4] = {};
    for (int bk = brow[I]; bk < brow[I + 1]; ++bk) {
        const int K = bcol[bk];
        const int b2 = find_block(bcol, brow[K], brow[K + 1], J);
        if (b2 >= brow[K + 1] || bcol[b2] != J) continue;
        const int nK = atom_off[K + 1] - atom_off[K];
        const double* eik = Bv + asc_voff[bk];
        const double* ekj = Bv + asc_voff[b2];
        for (int a = 0; a < nI; ++a)
            for (int m = 0; m < nK; ++m) {
                const double x = eik[a * nK + m] - ((K == I && a == m) ? 1.0 : 0.0);
                if (x == 0.0) continue;
                for (int c = 0; c < nJ; ++c) e2[a][c] += x * (ekj[m * nJ + c] - ((K == J && m == c) ? 1.0 : 0.0));
            }
    }
    for (int e = 0; e < 16; ++e) {
        const int a = e >> 2, c = e & 3;
        f[22 + e] = (a < nI && c < nJ) ? (float)(10.0 * e2[a][c]) : 0.f;
    }
    f[38] = I == J ? 1.f : 0.f;
    f[39] = 0.f;
}

void launch_spai_features(int64_t n, const int* pI, const int* pJ, const int* pb, const DevMatrix& d,
                          const int* bcol, const double* pos, double box, float* feat, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(spai_features_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, pI, pJ, pb,
                       d.atom_off, d.brow, bcol, d.asc_voff, d.B, pos, box, feat);
}

__global__ void eye_kernel(int M, int ld, int c0, double* __restrict__ S) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)M * ld) return;
    const int r = (int)(i / ld), c = (int)(i - (int64_t)r * ld);
    S[i] = (r == c0 + c) ? 1.0 : 0.0;
}

void launch_eye(int M, int ld, int c0, double* S, hipStream_t st) {
    const int64_t n = (int64_t)M * ld;
    hipLaunchKernelGGL(eye_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, M, ld, c0, S);
}

// target[p] = (B^{-1})_IJ for the pairs whose columns J's orbitals lie in
// [c0, c0 + ld) of X = B^{-1} [:, c0 : c0 + ld]  ([M][ld])
__global__ void spai_targets_kernel(int64_t n, const int* __restrict__ pI, const int* __restrict__ pJ,
                                    const int* __restrict__ atom_off, const double* __restrict__ X, int ld, int c0,
                                    float* __restrict__ target, float* __restrict__ mask) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int I = pI[p], J = pJ[p];
    const int oI = atom_off[I], oJ = atom_off[J];
    const int nI = atom_off[I + 1] - oI, nJ = atom_off[J + 1] - oJ;
    if (oJ < c0 || oJ + nJ > c0 + ld) return;
    for (int e = 0; e < 16; ++e) {
        const int a = e >> 2, c = e & 3;
        const bool ok = a < nI && c < nJ;
        target[p * 16 + e] = ok ? (float)X[(size_t)(oI + a) * ld + (oJ + c - c0)] : 0.f;
        mask[p * 16 + e] = ok ? 1.f : 0.f;
    }
}

void launch_spai_targets(int64_t n, const int* pI, const int* pJ, const int* atom_off, const double* X, int ld,
                         int c0, float* target, float* mask, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(spai_targets_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, pI, pJ,
                       atom_off, X, ld, c0, target, mask);
}

// ---------------------------------------------------------------------------
// FP32 training kernels
// ---------------------------------------------------------------------------

// C(i, j) (=, or += when acc) sum_k A(i, k) B(k, j) with A(i, k) = A[i sa0 + k sa1],
// B(k, j) = B[k sb0 + j sb1], C(i, j) = C[i sc0 + j], on the matrix cores
// (v_mfma_f32_16x16x4_f32, FP32 products and sums).  A workgroup of four
// waves owns a 64 x 64 tile of C; K goes in steps of 16 through LDS (zero
// outside the matrices); each wave computes a 32 x 32 quarter as 2 x 2
// blocks of 16 x 16.  Operand layout of the instruction: lane l supplies
// A(row l % 16, k l / 16) and B(k l / 16, column l % 16) and receives
// C(4 (l / 16) + i, l % 16), i = 0..3.
typedef float f32x4_mfma_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void gemm_kernel(int Mr, int N, int K, const float* __restrict__ A, int64_t sa0,
                                                   int64_t sa1, const float* __restrict__ B, int64_t sb0,
                                                   int64_t sb1, float* __restrict__ C, int64_t sc0, int acc) {
    __shared__ float As[16][68];
    __shared__ float Bs[16][68];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r16 = lane & 15, kq = lane >> 4;
    const int wi = (w >> 1) * 32, wj = (w & 1) * 32;  // the wave's quarter of the tile
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    f32x4_mfma_t c[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) c[bi][bj] = f32x4_mfma_t{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        for (int e = threadIdx.x; e < 64 * 16; e += 256) {
            const int ii = e >> 4, kk = e & 15;
            const int gi = i0 + ii, gk = k0 + kk;
            As[kk][ii] = (gi < Mr && gk < K) ? A[gi * sa0 + gk * sa1] : 0.f;
        }
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int kk = e >> 6, jj = e & 63;
            const int gk = k0 + kk, gj = j0 + jj;
            Bs[kk][jj] = (gk < K && gj < N) ? B[gk * sb0 + gj * sb1] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kk = 4 * ks + kq;
            const float a0 = As[kk][wi + r16], a1 = As[kk][wi + 16 + r16];
            const float b0 = Bs[kk][wj + r16], b1 = Bs[kk][wj + 16 + r16];
            c[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, c[0][0], 0, 0, 0);
            c[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, c[0][1], 0, 0, 0);
            c[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, c[1][0], 0, 0, 0);
            c[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, c[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gi = i0 + wi + 16 * bi + 4 * kq + q;
                const int gj = j0 + wj + 16 * bj + r16;
                if (gi >= Mr || gj >= N) continue;
                float* out = C + gi * sc0 + gj;
                *out = acc ? *out + c[bi][bj][q] : c[bi][bj][q];
            }
}

void launch_gemm(int Mr, int N, int K, const float* A, int64_t sa0, int64_t sa1, const float* B, int64_t sb0,
                 int64_t sb1, float* C, int64_t sc0, bool acc, hipStream_t st) {
    if (Mr <= 0 || N <= 0) return;
    hipLaunchKernelGGL(gemm_kernel, dim3((N + 63) / 64, (Mr + 63) / 64), dim3(256), 0, st, Mr, N, K, A, sa0, sa1, B,
                       sb0, sb1, C, sc0, acc ? 1 : 0);
}

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_df(float x) {
    return 0.5f * (1.f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// Z[i][j] += b[j]; H = act ? gelu(Z) : Z
__global__ void bias_act_kernel(int64_t rows, int N, float* __restrict__ Z, const float* __restrict__ b,
                                float* __restrict__ H, int act) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * N) return;
    const float z = Z[e] + b[e % N];
    Z[e] = z;
    H[e] = act ? gelu_f(z) : z;
}

void launch_bias_act(int64_t rows, int N, float* Z, const float* b, float* H, bool act, hipStream_t st) {
    const int64_t n = rows * N;
    if (n == 0) return;
    hipLaunchKernelGGL(bias_act_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rows, N, Z, b, H,
                       act ? 1 : 0);
}

__global__ void gelu_back_kernel(int64_t n, const float* __restrict__ Z, float* __restrict__ G) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) G[e] *= gelu_df(Z[e]);
}

void launch_gelu_back(int64_t n, const float* Z, float* G, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(gelu_back_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, Z, G);
}

// db[j] = sum_i G[i][j] (one thread per column, rows in order)
__global__ void colsum_kernel(int64_t rows, int N, const float* __restrict__ G, float* __restrict__ db) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.f;
    for (int64_t i = 0; i < rows; ++i) s += G[i * N + j];
    db[j] = s;
}

void launch_colsum(int64_t rows, int N, const float* G, float* db, hipStream_t st) {
    hipLaunchKernelGGL(colsum_kernel, dim3((N + 127) / 128), dim3(128), 0, st, rows, N, G, db);
}

// r = (out - T) W; partial sums of r^2 and W per block; gout = r (scaled later)
__global__ __launch_bounds__(256) void loss_partial_kernel(int64_t n, const float* __restrict__ out,
                                                           const float* __restrict__ T,
                                                           const float* __restrict__ W, float* __restrict__ gout,
                                                           double* __restrict__ part) {
    __shared__ double s1[256], s2[256];
    double a = 0.0, w = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const float r = (out[e] - T[e]) * W[e];
        gout[e] = r;
        a += (double)r * r;
        w += W[e];
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = w;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s1[threadIdx.x] += s1[threadIdx.x + o];
            s2[threadIdx.x] += s2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s1[0];
        part[2 * blockIdx.x + 1] = s2[0];
    }
}

// loss = sum r^2 / sum W; scale[0] = 2 / sum W (factor of the output gradient)
__global__ void loss_final_kernel(int nb, const double* __restrict__ part, double* __restrict__ loss,
                                  float* __restrict__ scale) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0, w = 0.0;
    for (int b = 0; b < nb; ++b) {
        a += part[2 * b];
        w += part[2 * b + 1];
    }
    *loss = w > 0.0 ? a / w : 0.0;
    *scale = w > 0.0 ? (float)(2.0 / w) : 0.f;
}

__global__ void scale_kernel(int64_t n, const float* __restrict__ scale, float* __restrict__ g) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) g[e] *= *scale;
}

constexpr int kLossBlocks = 64;

void launch_loss(int64_t n, const float* out, const float* T, const float* W, float* gout, double* part,
                 double* loss, float* scale, hipStream_t st) {
    hipLaunchKernelGGL(loss_partial_kernel, dim3(kLossBlocks), dim3(256), 0, st, n, out, T, W, gout, part);
    hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, st, kLossBlocks, part, loss, scale);
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, scale, gout);
}

__global__ void adam_kernel(int64_t n, float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    th[e] -= lr * (mm * c1) / (sqrtf(vv * c2) + eps);
}

void launch_adam(int64_t n, float* th, const float* g, float* m, float* v, float lr, int t, hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f / (1.f - powf(b1, (float)t)), c2 = 1.f / (1.f - powf(b2, (float)t));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, th, g, m, v, lr, b1, b2,
                       1e-8f, c1, c2);
}

__global__ void gather_rows_kernel(int n, int F, const int* __restrict__ idx, const float* __restrict__ src,
                                   float* __restrict__ dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * F) return;
    const int i = (int)(e / F), f = (int)(e - (int64_t)i * F);
    dst[e] = src[(int64_t)idx[i] * F + f];
}

void launch_gather_rows(int n, int F, const int* idx, const float* src, float* dst, hipStream_t st) {
    const int64_t t = (int64_t)n * F;
    if (t == 0) return;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, n, F, idx, src, dst);
}

// ---------------------------------------------------------------------------
// BF16 inference: weights and activations rounded to bfloat16 (round to
// nearest even), products accumulated in FP32, FP32 biases.
// ---------------------------------------------------------------------------

__device__ __forceinline__ float bf16_round(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}

__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__global__ void to_bf16_kernel(int64_t n, const float* __restrict__ x, uint16_t* __restrict__ y) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) y[e] = (uint16_t)(__float_as_uint(bf16_round(x[e])) >> 16);
}

void launch_to_bf16(int64_t n, const float* x, uint16_t* y, hipStream_t st) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, x, y);
}

// BF16 inference on the matrix cores: v_mfma_f32_16x16x32_bf16, FP32
// accumulation.  A workgroup of four waves stages the four weight matrices
// once in LDS (BF16 rows padded by 16 bytes against bank conflicts; layer 1's
// 40 inputs zero-padded to 64), then every wave runs tiles of 32 pairs
// through the four layers on its own, looping over tiles with a grid stride.
// Between layers a tile's activations live in the wave's LDS tile
// ([32][128] BF16); each layer's 16 x 16 output blocks are finished in
// registers (bias, GELU, BF16 rounding) and written back.  Operand layout
// of the instruction: lane l supplies row l % 16 of A and column l % 16 of B,
// each as the 8 consecutive k of k-group l / 16 (the same group for A and
// B), and receives D[4 (l / 16) + i][l % 16], i = 0..3.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kIW = 4;        // waves per workgroup
constexpr int kTP = 32;       // pairs per wave tile (two 16-row blocks)
constexpr int kS1 = 64 + 8;   // LDS row stride (BF16 elements) of W1
constexpr int kSH = 128 + 8;  // LDS row stride of W2, W3, W4 and of the activation tile

__device__ __forceinline__ uint16_t bf16_bits(float x) { return (uint16_t)(__float_as_uint(bf16_round(x)) >> 16); }

// 8 consecutive BF16 values (16-byte aligned) as one MFMA operand
__device__ __forceinline__ bf16x8_t ld_frag(const uint16_t* p) {
    return __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const uint4*>(p));
}

// acc[mt][nt] = sum over KS k-steps of 32: A block mt (rows of the tile) times
// W^T block nt (W rows 16 nt .. 16 nt + 15, row stride ws in LDS)
template <int KS, int NT>
__device__ __forceinline__ void mfma_layer(const bf16x8_t (&a)[2][KS], const uint16_t* W, int ws, int lane,
                                           f32x4_t (&acc)[2][NT]) {
    const int r16 = lane & 15, kg = lane >> 4;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        acc[0][nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        acc[1][nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const bf16x8_t b = ld_frag(W + (16 * nt + r16) * ws + 32 * ks + 8 * kg);
            acc[0][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][ks], b, acc[0][nt], 0, 0, 0);
            acc[1][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][ks], b, acc[1][nt], 0, 0, 0);
        }
    }
}

// hidden activations of a tile: H[row][n] = bf16(gelu(acc + b[n]))
__device__ __forceinline__ void store_hidden(const f32x4_t (&acc)[2][8], const float* __restrict__ b, uint16_t* H,
                                             int lane) {
    const int r16 = lane & 15, kg = lane >> 4;
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) {
        const float bb = b[16 * nt + r16];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                H[(16 * mt + 4 * kg + i) * kSH + 16 * nt + r16] = bf16_bits(gelu_f(acc[mt][nt][i] + bb));
    }
}

__device__ __forceinline__ void load_hidden(const uint16_t* H, int lane, bf16x8_t (&a)[2][4]) {
    const int r16 = lane & 15, kg = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) a[mt][ks] = ld_frag(H + (16 * mt + r16) * kSH + 32 * ks + 8 * kg);
}

__global__ __launch_bounds__(kIW * 64) void infer_mfma_kernel(int64_t n, const uint16_t* __restrict__ Wbf,
                                                               const float* __restrict__ params,
                                                               const float* __restrict__ feat,
                                                               float* __restrict__ out) {
    __shared__ __align__(16) uint16_t W1s[128 * kS1];
    __shared__ __align__(16) uint16_t W2s[128 * kSH];
    __shared__ __align__(16) uint16_t W3s[128 * kSH];
    __shared__ __align__(16) uint16_t W4s[16 * kSH];
    __shared__ __align__(16) uint16_t Hs[kIW][kTP * kSH];
    // offsets of the flat parameter layout (W1, b1, W2, b2, W3, b3, W4, b4)
    constexpr size_t oW1 = 0, ob1 = oW1 + 128 * 40, oW2 = ob1 + 128, ob2 = oW2 + 128 * 128, oW3 = ob2 + 128,
                     ob3 = oW3 + 128 * 128, oW4 = ob3 + 128, ob4 = oW4 + 16 * 128;
    for (int e = threadIdx.x; e < 128 * 64; e += blockDim.x) {
        const int r = e >> 6, c = e & 63;
        W1s[r * kS1 + c] = (c < 40) ? Wbf[oW1 + r * 40 + c] : (uint16_t)0;
    }
    for (int e = threadIdx.x; e < 128 * 128; e += blockDim.x) {
        const int r = e >> 7, c = e & 127;
        W2s[r * kSH + c] = Wbf[oW2 + e];
        W3s[r * kSH + c] = Wbf[oW3 + e];
    }
    for (int e = threadIdx.x; e < 16 * 128; e += blockDim.x) W4s[(e >> 7) * kSH + (e & 127)] = Wbf[oW4 + e];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r16 = lane & 15, kg = lane >> 4;
    uint16_t* H = Hs[w];
    const int64_t n_tiles = (n + kTP - 1) / kTP;
    for (int64_t t = (int64_t)blockIdx.x * kIW + w; t < n_tiles; t += (int64_t)gridDim.x * kIW) {
        const int64_t p0 = t * kTP;
        f32x4_t acc[2][8];
        {
            // layer 1 operands: the BF16-rounded features (k >= 40 and pairs past n are zero)
            bf16x8_t a[2][2];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const int64_t p = p0 + 16 * mt + r16;
                    const int k0 = 32 * ks + 8 * kg;
                    uint16_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                    if (p < n && k0 < 40) {
                        const float4 f0 = *reinterpret_cast<const float4*>(feat + p * 40 + k0);
                        const float4 f1 = *reinterpret_cast<const float4*>(feat + p * 40 + k0 + 4);
                        v[0] = bf16_bits(f0.x); v[1] = bf16_bits(f0.y); v[2] = bf16_bits(f0.z); v[3] = bf16_bits(f0.w);
                        v[4] = bf16_bits(f1.x); v[5] = bf16_bits(f1.y); v[6] = bf16_bits(f1.z); v[7] = bf16_bits(f1.w);
                    }
                    a[mt][ks] = __builtin_bit_cast(bf16x8_t, v);
                }
            mfma_layer<2, 8>(a, W1s, kS1, lane, acc);
        }
        // the wave's own tile: order its LDS writes and reads (lanes exchange rows through it)
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        store_hidden(acc, params + ob1, H, lane);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        for (int l = 0; l < 2; ++l) {
            bf16x8_t a[2][4];
            load_hidden(H, lane, a);
            mfma_layer<4, 8>(a, l == 0 ? W2s : W3s, kSH, lane, acc);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            store_hidden(acc, params + (l == 0 ? ob2 : ob3), H, lane);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        }
        bf16x8_t a[2][4];
        load_hidden(H, lane, a);
        f32x4_t o[2][1];
        mfma_layer<4, 1>(a, W4s, kSH, lane, o);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        const float bb = params[ob4 + r16];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t p = p0 + 16 * mt + 4 * kg + i;
                if (p < n) out[p * 16 + r16] = o[mt][0][i] + bb;
            }
    }
}

void launch_infer_bf16(int64_t n, const uint16_t* Wbf, const float* params, const float* feat, float* out,
                       hipStream_t st) {
    if (n == 0) return;
    int dev = 0, n_cu = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t n_tiles = (n + kTP - 1) / kTP;
    // one workgroup per CU holds the 127 KB of LDS; more would wait for it
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n_tiles + kIW - 1) / kIW, n_cu));
    hipLaunchKernelGGL(infer_mfma_kernel, dim3(grid), dim3(kIW * 64), 0, st, n, Wbf, params, feat, out);
}

// Assemble M on B's pattern (internal layout, FP64) from the upper-pair blocks:
// M_IJ = out_p (valid part), M_JI = M_IJ^T, diagonal blocks symmetrised.
__global__ void spai_assemble_kernel(int64_t n, const int* __restrict__ pI, const int* __restrict__ pJ,
                                     const int* __restrict__ pb, const int* __restrict__ pbt,
                                     const int* __restrict__ atom_off, const int64_t* __restrict__ asc_voff,
                                     const float* __restrict__ out, double* __restrict__ Mv) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int I = pI[p], J = pJ[p];
    const int nI = atom_off[I + 1] - atom_off[I], nJ = atom_off[J + 1] - atom_off[J];
    const float* o = out + p * 16;
    double* mij = Mv + asc_voff[pb[p]];
    double* mji = Mv + asc_voff[pbt[p]];
    for (int a = 0; a < nI; ++a)
        for (int c = 0; c < nJ; ++c) {
            double v = o[a * 4 + c];
            if (I == J) v = 0.5 * (v + (double)o[c * 4 + a]);
            mij[a * nJ + c] = v;
            if (I != J) mji[c * nI + a] = v;
        }
}

void launch_spai_assemble(int64_t n, const int* pI, const int* pJ, const int* pb, const int* pbt,
                          const DevMatrix& d, const float* out, double* Mv, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(spai_assemble_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, pI, pJ, pb, pbt,
                       d.atom_off, d.asc_voff, out, Mv);
}

}  // namespace elses
