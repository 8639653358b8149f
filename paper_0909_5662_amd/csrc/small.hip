// FP64 rotation of small blocks in one launch: O'_b = U^T (O_b (x) I_d) U
// (Sec. 2 step 5) for m <= 64 and m' <= 64, where the two-stage GEMM path
// is bound by launch latency (a 64-state batch is a few MFLOP per operator).
//
// One workgroup per (operator b, 16 output columns beta), four waves.  With
// U_s the m x m' matrix of U's rows j*d + s, the output is
//   O'_b = sum_s U_s^T (O_b U_s),
// taken site state by site state: T_s = O_b U_s[:, chunk] (m x 16) into LDS,
// then O'_b[:, chunk] += U_s^T T_s, every product on v_mfma_f64_16x16x4f64
// (lane l supplies A(row l%16, k l/16), B(k l/16, col l%16); accumulator
// element v of lane l is C(4v + l/16, l%16)).  O_b and U_s are staged in LDS
// zero-padded to 64 x 64, so partial extents need no guards in the products.
#include <hip/hip_runtime.h>

#include "rot_internal.h"

namespace rot {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kSmall = 64;       // largest m and m'
constexpr int kSmallPitch = 66;  // LDS row pitch (doubles): rows 4 banks apart
constexpr int kSmallCols = 16;   // output columns per workgroup

__global__ __launch_bounds__(256) void rotate_small_f64_kernel(const double* __restrict__ U, int64_t ldu,
                                                               const double* __restrict__ O, int64_t ldo,
                                                               int64_t stride_o, double* __restrict__ out,
                                                               int64_t ldout, int64_t stride_out, int m, int d,
                                                               int mp) {
    __shared__ double Os[kSmall * kSmallPitch];     // O_b[j][k]
    __shared__ double Us[2][kSmall * kSmallPitch];  // U_s[j][alpha], two site states in turn
    __shared__ double Ts[kSmall * kSmallCols];      // T_s[j][beta - beta0]
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int c = lane & 15, h = lane >> 4;
    const int b = blockIdx.y, beta0 = blockIdx.x * kSmallCols;
    const double* Ob = O + (int64_t)b * stride_o;
    constexpr int PER = kSmall * kSmall / 256;  // elements of a 64 x 64 tile per thread

    // Tile staging: thread tid owns column a = tid % 64 and rows j0 + 4 x
    // (j0 = tid / 64, x < PER).  Every load is unconditional, from a clamped
    // in-range row and column, so the loads stay in flight; entries outside
    // the block are replaced by zeros when the tile is stored to LDS.
    const int a = tid & (kSmall - 1), j0 = tid >> 6;
    const int ac = min(a, mp - 1), jb = min(j0, m - 1);
    const int xl = j0 < m ? (m - 1 - j0) >> 2 : 0;  // last x whose row exists
    auto keep = [&](int x, int cols) __attribute__((always_inline)) { return a < cols && j0 + 4 * x < m; };
    // U_s through registers: site state s + 1 is loaded while s is multiplied
    double ur[PER];
    const int64_t ustep = (int64_t)4 * d * ldu;  // four rows j further
    auto load_u = [&](int s) __attribute__((always_inline)) {
        const double* u0 = U + ((int64_t)jb * d + s) * ldu + ac;
        if (m == kSmall) {  // every row exists: addresses step by a uniform stride
#pragma unroll
            for (int x = 0; x < PER; x++) ur[x] = u0[x * ustep];
        } else {
            const double* ul = u0 + (int64_t)xl * ustep;
#pragma unroll
            for (int x = 0; x < PER; x++) ur[x] = *(x <= xl ? u0 + x * ustep : ul);
        }
    };
    auto store_u = [&](double* dst) __attribute__((always_inline)) {
#pragma unroll
        for (int x = 0; x < PER; x++) dst[(j0 + 4 * x) * kSmallPitch + a] = keep(x, mp) ? ur[x] : 0.0;
    };
    load_u(0);
    {
        double orr[PER];
        const double* o0 = Ob + (int64_t)jb * ldo + min(a, m - 1);
        const int64_t ostep = 4 * ldo;
        if (m == kSmall) {
#pragma unroll
            for (int x = 0; x < PER; x++) orr[x] = o0[x * ostep];
        } else {
            const double* ol = o0 + (int64_t)xl * ostep;
#pragma unroll
            for (int x = 0; x < PER; x++) orr[x] = *(x <= xl ? o0 + x * ostep : ol);
        }
#pragma unroll
        for (int x = 0; x < PER; x++) Os[(j0 + 4 * x) * kSmallPitch + a] = keep(x, m) ? orr[x] : 0.0;
    }
    store_u(Us[0]);
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < d; s++) {
        const double* us = Us[s & 1];
        if (s + 1 < d) load_u(s + 1);
        __syncthreads();  // U_s stored; the previous T_s consumed
        // T_s rows 16 w .. 16 w + 15 over the 16 columns of this chunk
        f64x4 t = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < kSmall / 4; q++) {
            const int k = 4 * q + h;
            t = __builtin_amdgcn_mfma_f64_16x16x4f64(Os[(16 * w + c) * kSmallPitch + k],
                                                    us[k * kSmallPitch + beta0 + c], t, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; v++) Ts[(16 * w + 4 * v + h) * kSmallCols + c] = t[v];
        __syncthreads();
        // O'_b rows alpha = 16 w .. 16 w + 15 += U_s^T T_s
#pragma unroll
        for (int q = 0; q < kSmall / 4; q++) {
            const int j = 4 * q + h;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(us[j * kSmallPitch + 16 * w + c], Ts[j * kSmallCols + c], acc,
                                                      0, 0, 0);
        }
        // the other buffer was last read in step s - 1, before this step's first barrier
        if (s + 1 < d) store_u(Us[(s + 1) & 1]);
    }
    double* ob = out + (int64_t)b * stride_out;
    const int beta = beta0 + c;
    if (beta < mp) {
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int alpha = 16 * w + 4 * v + h;
            if (alpha < mp) ob[(int64_t)alpha * ldout + beta] = acc[v];
        }
    }
}

}  // namespace

bool rotate_small_f64_applies(const rot_problem& p) {
    return p.m <= kSmall && p.mp <= kSmall && p.n_ops <= 65535 && p.m > 0 && p.mp > 0 && p.d > 0;
}

hipError_t rotate_small_f64(const rot_problem& p, hipStream_t stream) {
    if (p.n_ops == 0) return hipSuccess;
    if (!rotate_small_f64_applies(p)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((p.mp + kSmallCols - 1) / kSmallCols), (unsigned)p.n_ops);
    hipLaunchKernelGGL(rotate_small_f64_kernel, grid, dim3(256), 0, stream, static_cast<const double*>(p.U), p.ldu,
                       static_cast<const double*>(p.O), p.ldo, p.stride_o, static_cast<double*>(p.out), p.ldout,
                       p.stride_out, p.m, p.d, p.mp);
    return hipGetLastError();
}

}  // namespace rot
