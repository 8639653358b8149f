// Device helpers shared by the LDS-staged GEMM kernels (gemm.hip,
// grouped.hip, gemm_bf16x3.hip): the XCD-aware workgroup order and the
// operand slice staged through registers into LDS.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rot {
namespace {  // internal to each kernel file, like the kernels that use them

// XCD-aware workgroup order: hardware places workgroup id w on XCD w % 8;
// the returned linear id gives each XCD a contiguous range of tiles, so
// tiles sharing an operand panel stay on one XCD's L2.
__device__ inline int xcd_linear_id() {
    const int nwg = gridDim.x, wg = blockIdx.x;
    const int per = nwg / 8, rem = nwg % 8;
    const int xcd = wg % 8, idx = wg / 8;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); };

// One operand slice of R rows (M or N extent) by SK = 16 k-columns, copied by
// NT threads in 16-byte chunks from global memory through registers into
// LDS, in the orientation it has in global memory.
//
// K-contiguous rows are SK elements unpadded: NQ 16-byte chunks (4 for FP32,
// 8 for FP64), RPB = 16 / NQ rows per 256 bytes, chunk q of row r stored in
// slot q ^ ((r / RPB) % NQ).  The stores of 16 lanes (RPB rows x NQ chunks)
// and the fragment reads of 16 lanes (16 rows, one chunk) then each cover all
// 64 LDS banks once.  M/N-contiguous slices are rows of R + 4 elements.
template <typename T, int R, int NT, bool KCONTIG>
struct LdsSlice {
    typedef typename Vec16<T>::type V;
    static constexpr int SK = 16;
    static constexpr int PAD = 4;
    static constexpr int VW = 16 / sizeof(T);
    static constexpr int CHUNKS = R * SK / VW / NT;
    static_assert(CHUNKS >= 1 && CHUNKS * NT * VW == R * SK, "slice must split evenly over threads");
    static constexpr int NQ = SK / VW;
    static constexpr int RPB = 16 / NQ;
    static constexpr int PITCH = KCONTIG ? SK : (R + PAD);
    static constexpr int ELEMS = KCONTIG ? R * PITCH : SK * PITCH;
    V r[CHUNKS];

    // element offset of 16-byte chunk q (k = q*VW ..) of row `row` in a
    // K-contiguous slice
    __device__ static inline int kc_off(int row, int q) { return row * PITCH + (q ^ ((row / RPB) % NQ)) * VW; }

    // base points at element (row 0, k 0) of the operand; rows/ks are the
    // operand's full extents; r0/k0 the slice origin.  With VEC and `vec`
    // (16-byte aligned rows, known at compile time or per problem), a slice
    // wholly inside the operand (uniform over the workgroup) takes
    // unconditional vector loads, all in flight together; other slices load
    // element by element with bounds checks.
    template <bool VEC>
    __device__ inline void load(const T* __restrict__ base, int64_t ld, int r0, int rows, int k0, int ks, bool vec,
                                int tid) {
        const bool interior = VEC && vec && r0 + R <= rows && k0 + SK <= ks;
        if (interior) {
#pragma unroll
            for (int c = 0; c < CHUNKS; c++) {
                const int f = tid + c * NT;
                const int row = KCONTIG ? f / NQ : (f % (R / VW)) * VW;
                const int k = KCONTIG ? (f % NQ) * VW : f / (R / VW);
                const T* p = KCONTIG ? base + (int64_t)(r0 + row) * ld + k0 + k : base + (int64_t)(k0 + k) * ld + r0 + row;
                r[c] = *reinterpret_cast<const V*>(p);
            }
            return;
        }
#pragma unroll
        for (int c = 0; c < CHUNKS; c++) {
            const int f = tid + c * NT;
            int row, k;
            if (KCONTIG) {
                row = f / NQ;
                k = (f % NQ) * VW;
            } else {
                k = f / (R / VW);
                row = (f % (R / VW)) * VW;
            }
            const int gr = r0 + row, gk = k0 + k;
            const T* p = KCONTIG ? base + (int64_t)gr * ld + gk : base + (int64_t)gk * ld + gr;
#pragma unroll
            for (int e = 0; e < VW; e++) {
                const bool ok = KCONTIG ? (gr < rows && gk + e < ks) : (gk < ks && gr + e < rows);
                r[c][e] = ok ? p[e] : T(0);
            }
        }
    }
    __device__ inline void store(T* lds, int tid) const {
#pragma unroll
        for (int c = 0; c < CHUNKS; c++) {
            const int f = tid + c * NT;
            int off;
            if (KCONTIG) {
                off = kc_off(f / NQ, f % NQ);
            } else {
                off = (f / (R / VW)) * PITCH + (f % (R / VW)) * VW;
            }
            *reinterpret_cast<V*>(lds + off) = r[c];
        }
    }
};

}  // namespace
}  // namespace rot
