// Superblock measurements in FP64 (one-point values of block operators and
// products of operators of the two blocks): the reductions that follow the
// products done by the GEMM kernels.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rot_internal.h"

namespace rot {
namespace {

constexpr int kDotParts = 8;

// partial[b][p] = sum over elements e = p*256*... of Z_b[e] * rho[e] in FP64:
// workgroup (p, b) takes the strided elements tid + 256*(p + kDotParts*q).
template <typename T>
__global__ __launch_bounds__(256) void dot_partial_kernel(const T* __restrict__ Z, int64_t stride_z, int64_t n,
                                                          const double* __restrict__ rho, double* __restrict__ partial) {
    __shared__ double red[256];
    const int p = blockIdx.x, b = blockIdx.y;
    const T* z = Z + (int64_t)b * stride_z;
    double acc = 0.0;
    for (int64_t e = (int64_t)p * 256 + threadIdx.x; e < n; e += (int64_t)kDotParts * 256)
        acc += (double)z[e] * rho[e];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)b * kDotParts + p] = red[0];
}

__global__ void dot_final_kernel(const double* __restrict__ partial, int n_ops, double* __restrict__ e) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_ops) return;
    double acc = 0.0;
    for (int p = 0; p < kDotParts; p++) acc += partial[(int64_t)b * kDotParts + p];
    e[b] = acc;
}

// q_b[j][j'] = sum_s Q_b[s*mR + j][s*mR + j'] (Q_b of side dR*mR at
// Q + b*q_stride, q_b of side mR)
__global__ __launch_bounds__(256) void partial_trace_kernel(const double* __restrict__ Q, int64_t q_stride, int mR,
                                                            int dR, double* __restrict__ q) {
    const int64_t side = (int64_t)dR * mR, n = (int64_t)mR * mR;
    const int b = blockIdx.y;
    const double* Qb = Q + (int64_t)b * q_stride;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int64_t j = e / mR, jp = e % mR;
        double acc = 0.0;
        for (int s = 0; s < dR; s++) acc += Qb[((int64_t)s * mR + j) * side + (int64_t)s * mR + jp];
        q[(int64_t)b * n + e] = acc;
    }
}

}  // namespace

size_t expect_dot_scratch(int n_ops) { return (size_t)n_ops * kDotParts * sizeof(double); }

hipError_t expect_dots(const void* Z, bool z_double, int64_t stride_z, int64_t n, int n_ops, const double* rho,
                       double* partial, double* e, hipStream_t s) {
    if (n_ops <= 0) return hipSuccess;
    const dim3 grid(kDotParts, (unsigned)n_ops);
    if (z_double)
        hipLaunchKernelGGL(dot_partial_kernel<double>, grid, dim3(256), 0, s, static_cast<const double*>(Z), stride_z,
                           n, rho, partial);
    else
        hipLaunchKernelGGL(dot_partial_kernel<float>, grid, dim3(256), 0, s, static_cast<const float*>(Z), stride_z, n,
                           rho, partial);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(dot_final_kernel, dim3((unsigned)((n_ops + 255) / 256)), dim3(256), 0, s, partial, n_ops, e);
    return hipGetLastError();
}

hipError_t partial_trace(const double* Q, int64_t q_stride, int mR, int dR, int n_ops, double* q, hipStream_t s) {
    if (n_ops <= 0) return hipSuccess;
    const int64_t n = (int64_t)mR * mR;
    const dim3 grid((unsigned)std::min<int64_t>((n + 255) / 256, 1024), (unsigned)n_ops);
    hipLaunchKernelGGL(partial_trace_kernel, grid, dim3(256), 0, s, Q, q_stride, mR, dR, q);
    return hipGetLastError();
}

}  // namespace rot
