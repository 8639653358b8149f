// Element-wise utilities: the split-BF16 operand format (x = hi + lo with
// hi = bf16(x), lo = bf16(x - hi), both rounded to nearest even; x - hi is
// exact in FP32) and a zero-fill kernel that is safe under stream capture.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rot_internal.h"

namespace rot {
namespace {

// FP32 -> BF16 round to nearest even (the hardware conversion,
// v_cvt_pk_bf16_f32), as a bit pattern.
__device__ inline uint16_t rne_bf16(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__global__ void split_kernel(const float* __restrict__ x, int64_t n, uint16_t* __restrict__ hi,
                             uint16_t* __restrict__ lo) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = x[i];
    const uint16_t h = rne_bf16(v);
    hi[i] = h;
    lo[i] = rne_bf16(v - bf16_to_f32(h));
}

__global__ void zero_kernel(uint32_t* __restrict__ p, int64_t words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void zero_bytes_kernel(unsigned char* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// dst[i] = (accumulate ? dst[i] : 0) + part_0[i] + part_1[i] + ... in that
// fixed order (parts `stride` elements apart), so split-K results do not
// depend on scheduling.
template <typename T>
__global__ void sum_parts_kernel(T* __restrict__ dst, const T* __restrict__ src, int64_t n, int parts,
                                 int64_t stride, bool accumulate) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        T acc = accumulate ? dst[i] : T(0);
        for (int p = 0; p < parts; p++) acc += src[i + p * stride];
        dst[i] = acc;
    }
}

// dst[b][r][c] (row stride ld, matrix stride bs) = sum over p of
// src[p*pstride + (b*rows + r)*cols + c], in ascending p (deterministic).
template <typename T>
__global__ void sum_parts_2d_kernel(T* __restrict__ dst, int64_t ld, int64_t bs, const T* __restrict__ src, int rows,
                                    int cols, int64_t n, int parts, int64_t pstride) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / ((int64_t)rows * cols);
        const int64_t rc = i - b * rows * cols;
        const int64_t r = rc / cols, c = rc - r * cols;
        T acc = T(0);
        for (int p = 0; p < parts; p++) acc += src[i + p * pstride];
        dst[b * bs + r * ld + c] = acc;
    }
}

}  // namespace

hipError_t sum_parts_2d(void* dst, int64_t ld, int64_t bs, const void* src, int rows, int cols, int nmat, int parts,
                        int64_t pstride, bool is_double, hipStream_t stream) {
    const int64_t n = (int64_t)rows * cols * nmat;
    if (n <= 0) return hipSuccess;
    const dim3 grid((unsigned)std::min<int64_t>((n + 255) / 256, 8192));
    if (is_double)
        hipLaunchKernelGGL(sum_parts_2d_kernel<double>, grid, dim3(256), 0, stream, static_cast<double*>(dst), ld, bs,
                           static_cast<const double*>(src), rows, cols, n, parts, pstride);
    else
        hipLaunchKernelGGL(sum_parts_2d_kernel<float>, grid, dim3(256), 0, stream, static_cast<float*>(dst), ld, bs,
                           static_cast<const float*>(src), rows, cols, n, parts, pstride);
    return hipGetLastError();
}

hipError_t sum_parts(void* dst, const void* src, int64_t n, int parts, int64_t stride, bool accumulate,
                     bool is_double, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const dim3 grid((unsigned)std::min<int64_t>((n + 255) / 256, 8192));
    if (is_double)
        hipLaunchKernelGGL(sum_parts_kernel<double>, grid, dim3(256), 0, stream, static_cast<double*>(dst),
                           static_cast<const double*>(src), n, parts, stride, accumulate);
    else
        hipLaunchKernelGGL(sum_parts_kernel<float>, grid, dim3(256), 0, stream, static_cast<float*>(dst),
                           static_cast<const float*>(src), n, parts, stride, accumulate);
    return hipGetLastError();
}

hipError_t split_bf16(const float* x, int64_t n, uint16_t* hi, uint16_t* lo, hipStream_t stream) {
    hipLaunchKernelGGL(split_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, x, n, hi, lo);
    return hipGetLastError();
}

hipError_t fill_zero(void* p, int64_t bytes, hipStream_t stream) {
    if (bytes <= 0) return hipSuccess;
    if ((reinterpret_cast<uintptr_t>(p) & 3) == 0 && bytes % 4 == 0) {
        const int64_t words = bytes / 4;
        const int64_t blocks = std::min<int64_t>((words + 255) / 256, 4096);
        hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream,
                           static_cast<uint32_t*>(p), words);
    } else {
        hipLaunchKernelGGL(zero_bytes_kernel, dim3((unsigned)((bytes + 255) / 256)), dim3(256), 0, stream,
                           static_cast<unsigned char*>(p), bytes);
    }
    return hipGetLastError();
}

}  // namespace rot
