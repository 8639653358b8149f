// FP64 reductions on the GPU: the two-point expectation values of Eq. (11)
// summed over operator pairs, and the isometry deviation max|U^T U - I|.
// These are bandwidth/latency-bound passes (one read of each rotated
// operator); every sum is FP64 with a fixed order, so results are
// deterministic.
#include <hip/hip_runtime.h>

#include "rot_internal.h"

namespace rot {
namespace {

constexpr int kRowsPerBlock = 32;  // rows of one operator handled by a block

__device__ inline double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    return x;
}

// For operator b and a stripe of kRowsPerBlock rows a:
//   w[b][a]            = sum_c X_b[a,c] psi[c]          (X_b psi)
//   vpart[b][stripe][c] = sum_{a in stripe} X_b[a,c] psi[a]   (partial X_b^T psi)
// Block: 256 threads; each wave owns rows a = a0 + wave, a0 + wave + 4, ...
template <typename T>
__global__ __launch_bounds__(256) void psi_products(const T* __restrict__ X, int mp, int64_t stride,
                                                    const double* __restrict__ psi,
                                                    double* __restrict__ w,
                                                    double* __restrict__ vpart, int stripes) {
    const int b = blockIdx.y, stripe = blockIdx.x;
    const int a0 = stripe * kRowsPerBlock;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const T* Xb = X + (int64_t)b * stride;
    // row dot products, one wave per row
    for (int r = wave; r < kRowsPerBlock; r += 4) {
        const int a = a0 + r;
        if (a >= mp) break;
        double acc = 0.0;
        for (int c = lane; c < mp; c += 64) acc += (double)Xb[(int64_t)a * mp + c] * psi[c];
        acc = wave_sum(acc);
        if (lane == 0) w[(int64_t)b * mp + a] = acc;
    }
    // column partial sums over this stripe, one thread per column
    const int a_end = min(a0 + kRowsPerBlock, mp);
    for (int c = tid; c < mp; c += 256) {
        double acc = 0.0;
        for (int a = a0; a < a_end; a++) acc += (double)Xb[(int64_t)a * mp + c] * psi[a];
        vpart[((int64_t)b * stripes + stripe) * mp + c] = acc;
    }
}

// v[b][c] = sum over stripes (fixed order), one thread per (b, c)
__global__ void reduce_stripes(const double* __restrict__ vpart, double* __restrict__ v, int mp, int n_ops,
                               int stripes) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)mp * n_ops) return;
    const int64_t b = idx / mp, c = idx % mp;
    double acc = 0.0;
    for (int s = 0; s < stripes; s++) acc += vpart[(b * stripes + s) * mp + c];
    v[idx] = acc;
}

// S_w = sum_b w_b, S_v = sum_b v_b (fixed order over b)
__global__ void sum_over_ops(const double* __restrict__ w, const double* __restrict__ v, double* __restrict__ sw,
                             double* __restrict__ sv, int mp, int n_ops) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= mp) return;
    double tw = 0.0, tv = 0.0;
    for (int b = 0; b < n_ops; b++) {
        tw += w[(int64_t)b * mp + c];
        tv += v[(int64_t)b * mp + c];
    }
    sw[c] = tw;
    sv[c] = tv;
}

// pairs[i][j] = v_i . w_j, one block per (i, j)
__global__ __launch_bounds__(256) void pair_dots(const double* __restrict__ v,
                                                 const double* __restrict__ w,
                                                 double* __restrict__ pairs, int mp, int n_ops) {
    const int i = blockIdx.y, j = blockIdx.x;
    __shared__ double red[4];
    double acc = 0.0;
    for (int a = threadIdx.x; a < mp; a += 256) acc += v[(int64_t)i * mp + a] * w[(int64_t)j * mp + a];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) pairs[(int64_t)i * n_ops + j] = ((red[0] + red[1]) + red[2]) + red[3];
}

// loss = S_v . S_w  (= sum_ij v_i . w_j), single block
__global__ __launch_bounds__(256) void loss_dot(const double* __restrict__ sv,
                                                const double* __restrict__ sw, double* loss, int mp) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int a = threadIdx.x; a < mp; a += 256) acc += sv[a] * sw[a];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) *loss = ((red[0] + red[1]) + red[2]) + red[3];
}

// grad[a][c] = psi[a] S_w[c] + S_v[a] psi[c]
template <typename T>
__global__ void loss_grad(const double* __restrict__ psi, const double* __restrict__ sw,
                          const double* __restrict__ sv, T* __restrict__ grad, int mp) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)mp * mp) return;
    const int a = (int)(idx / mp), c = (int)(idx % mp);
    grad[idx] = (T)(psi[a] * sw[c] + sv[a] * psi[c]);
}

// y (rows x cols, packed) = x (rows x cols, row stride ld) widened to FP64
template <typename T>
__global__ void widen(const T* __restrict__ x, int64_t ld, int cols, double* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (double)x[(i / cols) * ld + i % cols];
}

// max that keeps a NaN from either side (fmax would drop it, and a U with a
// NaN entry would then pass the isometry check)
__device__ inline double max_keep_nan(double a, double b) { return (b > a || b != b) ? b : a; }

// partial[block] = max |G[a][b] - delta_ab| over a grid-stride range
__global__ __launch_bounds__(256) void max_dev_partial(const double* __restrict__ G, int cols,
                                                       double* __restrict__ partial) {
    const int64_t n = (int64_t)cols * cols;
    double worst = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int64_t a = i / cols, b = i % cols;
        worst = max_keep_nan(worst, fabs(G[i] - (a == b ? 1.0 : 0.0)));
    }
    __shared__ double red[256];
    red[threadIdx.x] = worst;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = max_keep_nan(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void max_final(const double* __restrict__ partial, int n, double* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double worst = 0.0;
        for (int i = 0; i < n; i++) worst = max_keep_nan(worst, partial[i]);
        *out = worst;
    }
}

}  // namespace

constexpr int kDevBlocks = 512;

size_t pair_loss_workspace_bytes(int mp, int n_ops) {
    const int stripes = (mp + kRowsPerBlock - 1) / kRowsPerBlock;
    const size_t vec = (size_t)mp * n_ops;
    return sizeof(double) * (vec * 2 + vec * stripes + 2 * (size_t)mp);
}

hipError_t pair_loss(const void* X, int mp, int n_ops, int64_t stride, bool is_double,
                     const double* psi, double* loss, double* pairs, void* grad, void* ws,
                     hipStream_t stream) {
    const int stripes = (mp + kRowsPerBlock - 1) / kRowsPerBlock;
    double* w = static_cast<double*>(ws);
    double* v = w + (size_t)mp * n_ops;
    double* vpart = v + (size_t)mp * n_ops;
    double* sw = vpart + (size_t)mp * n_ops * stripes;
    double* sv = sw + mp;
    const dim3 g1(stripes, n_ops);
    if (is_double)
        hipLaunchKernelGGL(psi_products<double>, g1, dim3(256), 0, stream,
                           static_cast<const double*>(X), mp, stride, psi, w, vpart, stripes);
    else
        hipLaunchKernelGGL(psi_products<float>, g1, dim3(256), 0, stream,
                           static_cast<const float*>(X), mp, stride, psi, w, vpart, stripes);
    const int64_t nv = (int64_t)mp * n_ops;
    hipLaunchKernelGGL(reduce_stripes, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, stream, vpart, v, mp,
                       n_ops, stripes);
    hipLaunchKernelGGL(sum_over_ops, dim3((mp + 255) / 256), dim3(256), 0, stream, w, v, sw, sv, mp, n_ops);
    if (pairs)
        hipLaunchKernelGGL(pair_dots, dim3(n_ops, n_ops), dim3(256), 0, stream, v, w, pairs, mp, n_ops);
    hipLaunchKernelGGL(loss_dot, dim3(1), dim3(256), 0, stream, sv, sw, loss, mp);
    if (grad) {
        const int64_t n = (int64_t)mp * mp;
        const dim3 gg((unsigned)((n + 255) / 256));
        if (is_double)
            hipLaunchKernelGGL(loss_grad<double>, gg, dim3(256), 0, stream, psi, sw, sv,
                               static_cast<double*>(grad), mp);
        else
            hipLaunchKernelGGL(loss_grad<float>, gg, dim3(256), 0, stream, psi, sw, sv,
                               static_cast<float*>(grad), mp);
    }
    return hipGetLastError();
}

static inline size_t round256(size_t n) { return (n + 31) / 32 * 32; }  // in doubles

// Workspace layout (doubles): [0] result, [32..32+kDevBlocks) partial maxima,
// then G = U^T U (cols x cols), then (float U only) U widened to FP64.
size_t isometry_workspace_bytes(int64_t rows, int cols, bool is_double) {
    size_t n = 32 + round256(kDevBlocks) + round256((size_t)cols * cols);
    if (!is_double) n += round256((size_t)rows * cols);
    return n * sizeof(double);
}

// G = U^T U in FP64 (matrix cores), then max |G - I| into ws[0].
hipError_t isometry_deviation(const void* U, int rows, int cols, int64_t ldu, bool is_double, double* ws,
                              hipStream_t stream) {
    double* dev = ws;
    double* partial = ws + 32;
    double* G = partial + round256(kDevBlocks);
    double* Ud = G + round256((size_t)cols * cols);
    const double* src = static_cast<const double*>(U);
    int64_t ld = ldu;
    if (!is_double) {
        const int64_t n = (int64_t)rows * cols;
        hipLaunchKernelGGL(widen<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                           static_cast<const float*>(U), ldu, cols, Ud, n);
        src = Ud;
        ld = cols;
    }
    GemmDesc g{};
    g.M = cols; g.N = cols; g.K = rows; g.batch = 1; g.kbatch = 1;
    g.A = src; g.lda = ld; g.a_kcontig = false;  // A(a, r) = U[r][a]
    g.B = src; g.ldb = ld; g.b_kcontig = false;  // B(r, b) = U[r][b]
    g.C = G; g.ldc = cols;
    hipError_t e = gemm_f64(g, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(max_dev_partial, dim3(kDevBlocks), dim3(256), 0, stream, G, cols, partial);
    hipLaunchKernelGGL(max_final, dim3(1), dim3(64), 0, stream, partial, kDevBlocks, dev);
    return hipGetLastError();
}

}  // namespace rot
