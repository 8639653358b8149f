// Device helpers shared by the LDS-staged GEMM kernels (gemm.hip,
// grouped.hip, gemm_bf16x3.hip): the XCD-aware workgroup order, the operand
// slice staged through registers into LDS, and (gemm.hip) the FP32 slice
// filled by buffer loads with LDS destination.
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

// One FP32 K slice (16 k) of 128 rows (M/N extent) filled by buffer loads
// with LDS destination, for a workgroup of 4 waves: no staging registers and
// no per-slice address arithmetic (the slice advance is the scalar offset).
// Wave w copies 1 KB pieces w and w + 4, lane l the 16 bytes at piece offset
// 16 l.  LDS layouts:
//  * K-contiguous operand: 128 rows of 16 floats, chunk q of row r in slot
//    q ^ ((r / 4) % 4) (LdsSlice<float, 128, ., true>::kc_off); piece y holds
//    rows 16 y .. 16 y + 15, so lane l fetches row 16 y + l / 4, chunk
//    (l % 4) ^ ((row / 4) % 4).
//  * M/N-contiguous operand: k rows of 128 floats in pairs, pair p (rows 2p,
//    2p + 1, one piece) at 264 p floats: rows k and k + 8, which the fragment
//    reads of the two lane halves take together, then lie 32 banks apart.
// Both take as many floats as the LdsSlice layouts of the same slice.  The
// operand's byte offsets (from the descriptor's base) must stay below 2^32.
template <bool KCONTIG>
struct DmaSlice128 {
    static constexpr int R = 128, SK = 16, PAIR = 2 * R + 8;
    static constexpr int ELEMS = KCONTIG ? R * SK : (SK / 2) * PAIR;
    uint32_t off[2];  // this lane's byte offsets in its two pieces of slice 0
    uint32_t step;    // bytes from one slice to the next

    __device__ static inline int kc_off(int row, int q) { return row * SK + (q ^ ((row >> 2) & 3)) * 4; }
    __device__ static inline int mn_off(int kr, int col) { return (kr >> 1) * PAIR + (kr & 1) * R + col; }
    __device__ static inline int piece(int y) { return KCONTIG ? y * 256 : y * PAIR; }

    // ld: the operand's row stride (elements); r0: the slice's first row (M/N)
    __device__ inline void init(int64_t ld, int r0, int wave, int lane) {
#pragma unroll
        for (int x = 0; x < 2; x++) {
            const int y = wave + 4 * x;
            int64_t e;
            if (KCONTIG) {
                const int row = 16 * y + (lane >> 2);
                e = (int64_t)(r0 + row) * ld + 4 * ((lane & 3) ^ ((row >> 2) & 3));
            } else {
                e = (int64_t)(2 * y + (lane >> 5)) * ld + r0 + 4 * (lane & 31);
            }
            off[x] = (uint32_t)(e * 4);
        }
        step = (uint32_t)(KCONTIG ? SK * 4 : (int64_t)SK * ld * 4);
    }
    // the slice `soff` bytes past slice 0 of the operand behind `rs` into
    // `buf` (ELEMS floats of LDS)
    __device__ inline void issue_at(__amdgpu_buffer_rsrc_t rs, float* buf, uint32_t soff, int wave) const {
        typedef __attribute__((address_space(3))) void* lptr;
#pragma unroll
        for (int x = 0; x < 2; x++)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lptr)(buf + piece(wave + 4 * x)), 16, off[x], (int)soff, 0, 0);
    }
    // slice t
    __device__ inline void issue(__amdgpu_buffer_rsrc_t rs, float* buf, int t, int wave) const {
        issue_at(rs, buf, (uint32_t)t * step, wave);
    }
};

// The FP64 counterpart for a workgroup of 4 waves: 128 rows by 16 doubles,
// 16 pieces of 1 KB, wave w copying pieces w, w + 4, w + 8, w + 12, in the
// layouts of LdsSlice<double, 128, ., K>: a K-contiguous slice holds 8 rows
// per piece (chunk q of row r in slot q ^ ((r / 2) % 8)), an M/N-contiguous
// one a k row of 128 doubles per piece at a pitch of 132.
template <bool KCONTIG>
struct DmaSlice128D {
    static constexpr int R = 128, SK = 16, PITCH = KCONTIG ? SK : R + 4;
    static constexpr int ELEMS = KCONTIG ? R * SK : SK * PITCH;
    uint32_t off[4];
    uint32_t step;

    __device__ static inline int piece(int y) { return KCONTIG ? y * 128 : y * PITCH; }
    __device__ inline void init(int64_t ld, int r0, int wave, int lane) {
#pragma unroll
        for (int x = 0; x < 4; x++) {
            const int y = wave + 4 * x;
            int64_t e;
            if (KCONTIG) {
                const int row = 8 * y + (lane >> 3);
                e = (int64_t)(r0 + row) * ld + 2 * ((lane & 7) ^ ((row >> 1) & 7));
            } else {
                e = (int64_t)y * ld + r0 + 2 * lane;
            }
            off[x] = (uint32_t)(e * 8);
        }
        step = (uint32_t)(KCONTIG ? SK * 8 : (int64_t)SK * ld * 8);
    }
    __device__ inline void issue_at(__amdgpu_buffer_rsrc_t rs, double* buf, uint32_t soff, int wave) const {
        typedef __attribute__((address_space(3))) void* lptr;
#pragma unroll
        for (int x = 0; x < 4; x++)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lptr)(buf + piece(wave + 4 * x)), 16, off[x], (int)soff, 0, 0);
    }
};

// Wait until this wave's buffer loads with LDS destination are done, then
// the workgroup barrier (the compiler neither moves memory accesses across
// it nor counts those loads itself).
__device__ inline void dma_slice_sync() {
    __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

}  // namespace
}  // namespace rot
