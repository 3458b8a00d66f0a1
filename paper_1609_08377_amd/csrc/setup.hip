// Setup kernels: the Lanczos sweep that brackets the spectrum of the overlap B
// (the overlap solve needs an interval [b_lo, b_hi] containing it), and
// small vector helpers.
#include "internal.h"

namespace elses {

// w <- w - a v - b u
__global__ void lanczos_orth_kernel(double* __restrict__ w, const double* __restrict__ v,
                                    const double* __restrict__ u, double a, double b, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w[i] = w[i] - a * v[i] - b * u[i];
}

// u <- v ; v <- w * s
__global__ void lanczos_shift_kernel(double* __restrict__ u, double* __restrict__ v, const double* __restrict__ w,
                                     double s, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        u[i] = v[i];
        v[i] = w[i] * s;
    }
}

void launch_lanczos_orth(double* w, const double* v, const double* u, double a, double b, int n, hipStream_t st) {
    hipLaunchKernelGGL(lanczos_orth_kernel, dim3((n + 255) / 256), dim3(256), 0, st, w, v, u, a, b, n);
}

void launch_lanczos_shift(double* u, double* v, const double* w, double s, int n, hipStream_t st) {
    hipLaunchKernelGGL(lanczos_shift_kernel, dim3((n + 255) / 256), dim3(256), 0, st, u, v, w, s, n);
}

}  // namespace elses
