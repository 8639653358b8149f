// Operators blocked together with the added site, out = U^T (X (x) S) U:
// the sum over the site index is folded into the stage-2 operand,
//   U'[(i,t), alpha] = x_i sum_s S[s,t] U[(i,s), alpha]  =  ((diag(x) (x) S^T) U)[(i,t), alpha],
// so that out = U'^T (X U_r) for a dense block operator X and out = U'^T U
// for X = diag(x) (the identity when x is absent).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rot_internal.h"

namespace rot {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void site_mix_kernel(const T* __restrict__ U, int64_t rows, int d, int mp,
                                                       SiteMatrix S, const T* __restrict__ x, T* __restrict__ Up) {
    const int64_t n = rows * mp;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int64_t r = e / mp;
        const int a = (int)(e % mp);
        const int64_t i = r / d;
        const int t = (int)(r % d);
        const T* u = U + i * d * mp + a;  // U[(i, 0), a]
        T acc = T(0);
        for (int s = 0; s < d; s++) acc += (T)S.v[s * d + t] * u[(int64_t)s * mp];
        Up[e] = x ? x[i] * acc : acc;
    }
}

}  // namespace

hipError_t site_mix(const void* U, int m, int d, int mp, const SiteMatrix& S, const void* x, void* Up,
                    bool is_double, hipStream_t stream) {
    const int64_t rows = (int64_t)m * d;
    const int64_t n = rows * mp;
    if (n <= 0) return hipSuccess;
    const dim3 grid((unsigned)std::min<int64_t>((n + 255) / 256, 16384));
    if (is_double)
        hipLaunchKernelGGL(site_mix_kernel<double>, grid, dim3(256), 0, stream, static_cast<const double*>(U), rows,
                           d, mp, S, static_cast<const double*>(x), static_cast<double*>(Up));
    else
        hipLaunchKernelGGL(site_mix_kernel<float>, grid, dim3(256), 0, stream, static_cast<const float*>(U), rows,
                           d, mp, S, static_cast<const float*>(x), static_cast<float*>(Up));
    return hipGetLastError();
}

}  // namespace rot
