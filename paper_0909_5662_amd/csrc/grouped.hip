// Grouped FP32 matrix-core GEMM over a work-list: one launch processes many
// independent GEMMs of different shapes (the quantum-number sector blocks of
// Eq. (10), or many rotations of different m in one sweep step).
//
// Each entry of the tile list names a problem and a C tile.  Workgroups are
// persistent: either a static schedule (workgroup w takes tiles w, w+G, ...,
// contiguous runs per XCD) or a dynamic queue (an atomic counter hands out
// the next tile, the GPU analogue of the paper's pool of tasks, Sec. 3.2).
// Every workgroup leaves the loop once the counter passes the last tile.
//
// Problem pointers are given as element offsets from per-launch base
// pointers, so a tile list built once for a block structure can be reused
// with new buffers; with a null base the offset is an absolute address.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "buffer_rsrc.h"
#include "lds_slice.h"
#include "rot_internal.h"

namespace rot {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kSlice = 16;  // K elements per LDS slice (LdsSlice::SK)

// BM x BN tile, WM x WN waves, each wave (BM/WM) x (BN/WN) made of 32 x 32
// blocks of v_mfma_f32_32x32x2f32 (lane layout as in gemm.hip).  Registers
// are capped for at least 3 waves per SIMD (the persistent loop's problem
// and tile state would otherwise take the 128 x 128 tile to 2).
template <int BM, int BN, int WM, int WN, bool AK, bool BK, bool DYN>
__global__ __launch_bounds__(WM* WN * 64) __attribute__((amdgpu_waves_per_eu(3))) void grouped_f32_kernel(
    GroupedLaunch L) {
    constexpr int NT = WM * WN * 64;
    constexpr int BI = BM / WM / 32, BJ = BN / WN / 32;
    typedef LdsSlice<float, BM, NT, AK> SA;
    typedef LdsSlice<float, BN, NT, BK> SB;
    __shared__ __attribute__((aligned(16))) float As[2][SA::ELEMS];
    __shared__ __attribute__((aligned(16))) float Bs[2][SB::ELEMS];
    __shared__ int s_next;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int h = lane >> 5, c = lane & 31;

    // first tile
    int t;
    if (DYN) {
        if (tid == 0) s_next = atomicAdd(L.counter, 1);
        __syncthreads();
        t = __builtin_amdgcn_readfirstlane(s_next);  // the same for every thread: keep it scalar
    } else {
        // static: contiguous runs per XCD (hardware puts workgroup w on XCD w % 8)
        const int nwg = gridDim.x, wg = blockIdx.x;
        const int per = nwg / 8, rem = nwg % 8, xcd = wg % 8, idx = wg / 8;
        t = xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
    }

    while (t < L.n_tiles) {
        const GroupedTile tile = L.tiles[t];
        const GroupedProblem p = L.probs[tile.prob];
        // null base: the offset is an absolute address
        const float* Ab = L.a_base ? L.a_base + p.a_off : reinterpret_cast<const float*>(p.a_off);
        const float* Bb = L.b_base ? L.b_base + p.b_off : reinterpret_cast<const float*>(p.b_off);
        const bool vec = p.flags & kGroupedVec;
        const int nk = (p.K + kSlice - 1) / kSlice;

        SA la;
        SB lb;
        f32x16 acc[BI][BJ];
#pragma unroll
        for (int i = 0; i < BI; i++)
#pragma unroll
            for (int j = 0; j < BJ; j++)
#pragma unroll
                for (int v = 0; v < 16; v++) acc[i][j][v] = 0.f;

        if (nk > 0) {
            la.template load<true>(Ab, p.lda, tile.m0, p.M, 0, p.K, vec, tid);
            lb.template load<true>(Bb, p.ldb, tile.n0, p.N, 0, p.K, vec, tid);
            la.store(As[0], tid);
            lb.store(Bs[0], tid);
        }
        __syncthreads();
        for (int kt = 0; kt < nk; kt++) {
            const int cur = kt & 1;
            if (kt + 1 < nk) {
                la.template load<true>(Ab, p.lda, tile.m0, p.M, (kt + 1) * kSlice, p.K, vec, tid);
                lb.template load<true>(Bb, p.ldb, tile.n0, p.N, (kt + 1) * kSlice, p.K, vec, tid);
            }
            const float* a_s = As[cur];
            const float* b_s = Bs[cur];
            float av[BI][8], bv[BJ][8];
#pragma unroll
            for (int i = 0; i < BI; i++) {
                const int row = wm * (BM / WM) + i * 32 + c;
                if (AK) {
                    const f32x4 x0 = *reinterpret_cast<const f32x4*>(a_s + SA::kc_off(row, 2 * h));
                    const f32x4 x1 = *reinterpret_cast<const f32x4*>(a_s + SA::kc_off(row, 2 * h + 1));
#pragma unroll
                    for (int e = 0; e < 4; e++) { av[i][e] = x0[e]; av[i][4 + e] = x1[e]; }
                } else {
#pragma unroll
                    for (int j = 0; j < 8; j++) av[i][j] = a_s[(h * 8 + j) * SA::PITCH + row];
                }
            }
#pragma unroll
            for (int i = 0; i < BJ; i++) {
                const int col = wn * (BN / WN) + i * 32 + c;
                if (BK) {
                    const f32x4 x0 = *reinterpret_cast<const f32x4*>(b_s + SB::kc_off(col, 2 * h));
                    const f32x4 x1 = *reinterpret_cast<const f32x4*>(b_s + SB::kc_off(col, 2 * h + 1));
#pragma unroll
                    for (int e = 0; e < 4; e++) { bv[i][e] = x0[e]; bv[i][4 + e] = x1[e]; }
                } else {
#pragma unroll
                    for (int j = 0; j < 8; j++) bv[i][j] = b_s[(h * 8 + j) * SB::PITCH + col];
                }
            }
#pragma unroll
            for (int j = 0; j < 8; j++)
#pragma unroll
                for (int i = 0; i < BI; i++)
#pragma unroll
                    for (int k = 0; k < BJ; k++)
                        acc[i][k] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i][j], bv[k][j], acc[i][k], 0, 0, 0);
            if (kt + 1 < nk) {
                la.store(As[cur ^ 1], tid);
                lb.store(Bs[cur ^ 1], tid);
            }
            __syncthreads();
        }

        float* Cb = L.c_base ? L.c_base + p.c_off : reinterpret_cast<float*>(p.c_off);
        const bool accum = p.flags & kGroupedAccumulate;
#pragma unroll
        for (int i = 0; i < BI; i++)
#pragma unroll
            for (int k = 0; k < BJ; k++) {
                const int col = tile.n0 + wn * (BN / WN) + k * 32 + c;
                if (col >= p.N) continue;
#pragma unroll
                for (int v = 0; v < 16; v++) {
                    const int row = tile.m0 + wm * (BM / WM) + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
                    if (row < p.M) {
                        float* q = Cb + (int64_t)row * p.ldc + col;
                        *q = accum ? *q + acc[i][k][v] : acc[i][k][v];
                    }
                }
            }

        if (DYN) {
            if (tid == 0) s_next = atomicAdd(L.counter, 1);
            __syncthreads();
            t = __builtin_amdgcn_readfirstlane(s_next);
            __syncthreads();  // everyone has read s_next before it is overwritten
        } else {
            t += gridDim.x;
        }
    }
}

// 128 x 128 tiles of whole problems (kGroupedWhole) with both K slices
// filled by buffer loads with LDS destination (DmaSlice128), four waves of
// 64 x 64: the persistent tile loop of grouped_f32_kernel around the K loop
// of the whole-tile GEMM kernel in gemm.hip (same fragment reads and
// products, so the same bits as the register-staged 128 x 128 shape).
template <bool AK, bool BK, bool DYN>
__global__ __launch_bounds__(256) void grouped_f32_dl_kernel(GroupedLaunch L) {
    typedef DmaSlice128<AK> DA;
    typedef DmaSlice128<BK> DB;
    __shared__ __attribute__((aligned(1024))) float As[2][DA::ELEMS];
    __shared__ __attribute__((aligned(1024))) float Bs[2][DB::ELEMS];
    __shared__ int s_next;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int h = lane >> 5, c = lane & 31;

    int t;
    if (DYN) {
        if (tid == 0) s_next = atomicAdd(L.counter, 1);
        __syncthreads();
        t = __builtin_amdgcn_readfirstlane(s_next);
    } else {
        const int nwg = gridDim.x, wg = blockIdx.x;
        const int per = nwg / 8, rem = nwg % 8, xcd = wg % 8, idx = wg / 8;
        t = xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
    }

    while (t < L.n_tiles) {
        const GroupedTile tile = L.tiles[t];
        const GroupedProblem p = L.probs[tile.prob];
        const float* Ab = L.a_base ? L.a_base + p.a_off : reinterpret_cast<const float*>(p.a_off);
        const float* Bb = L.b_base ? L.b_base + p.b_off : reinterpret_cast<const float*>(p.b_off);
        const __amdgpu_buffer_rsrc_t ra =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(Ab), (short)0, (int)0xffffffff, kBufferFlags);
        const __amdgpu_buffer_rsrc_t rb =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(Bb), (short)0, (int)0xffffffff, kBufferFlags);
        DA da;
        DB db;
        da.init(p.lda, tile.m0, wave, lane);
        db.init(p.ldb, tile.n0, wave, lane);
        const int nk = p.K / kSlice;

        f32x16 acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
            for (int j = 0; j < 2; j++)
#pragma unroll
                for (int v = 0; v < 16; v++) acc[i][j][v] = 0.f;

        da.issue(ra, As[0], 0, wave);
        db.issue(rb, Bs[0], 0, wave);
        dma_slice_sync();
        for (int kt = 0; kt < nk; kt++) {
            const int cur = kt & 1;
            if (kt + 1 < nk) {
                da.issue(ra, As[cur ^ 1], kt + 1, wave);
                db.issue(rb, Bs[cur ^ 1], kt + 1, wave);
            }
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            const float* a_s = As[cur];
            const float* b_s = Bs[cur];
            float av[2][8], bv[2][8];
#pragma unroll
            for (int i = 0; i < 2; i++) {
                const int row = wm * 64 + i * 32 + c;
                if (AK) {
                    const f32x4 x0 = *reinterpret_cast<const f32x4*>(a_s + DA::kc_off(row, 2 * h));
                    const f32x4 x1 = *reinterpret_cast<const f32x4*>(a_s + DA::kc_off(row, 2 * h + 1));
#pragma unroll
                    for (int e = 0; e < 4; e++) { av[i][e] = x0[e]; av[i][4 + e] = x1[e]; }
                } else {
#pragma unroll
                    for (int j = 0; j < 8; j++) av[i][j] = a_s[DA::mn_off(h * 8 + j, row)];
                }
            }
#pragma unroll
            for (int i = 0; i < 2; i++) {
                const int col = wn * 64 + i * 32 + c;
                if (BK) {
                    const f32x4 x0 = *reinterpret_cast<const f32x4*>(b_s + DB::kc_off(col, 2 * h));
                    const f32x4 x1 = *reinterpret_cast<const f32x4*>(b_s + DB::kc_off(col, 2 * h + 1));
#pragma unroll
                    for (int e = 0; e < 4; e++) { bv[i][e] = x0[e]; bv[i][4 + e] = x1[e]; }
                } else {
#pragma unroll
                    for (int j = 0; j < 8; j++) bv[i][j] = b_s[DB::mn_off(h * 8 + j, col)];
                }
            }
#pragma unroll
            for (int j = 0; j < 8; j++)
#pragma unroll
                for (int i = 0; i < 2; i++)
#pragma unroll
                    for (int k = 0; k < 2; k++)
                        acc[i][k] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i][j], bv[k][j], acc[i][k], 0, 0, 0);
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            dma_slice_sync();
        }

        float* Cb = L.c_base ? L.c_base + p.c_off : reinterpret_cast<float*>(p.c_off);
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
            for (int k = 0; k < 2; k++) {
                const int col = tile.n0 + wn * 64 + k * 32 + c;
#pragma unroll
                for (int v = 0; v < 16; v++) {
                    const int row = tile.m0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
                    Cb[(int64_t)row * p.ldc + col] = acc[i][k][v];
                }
            }

        if (DYN) {
            if (tid == 0) s_next = atomicAdd(L.counter, 1);
            __syncthreads();
            t = __builtin_amdgcn_readfirstlane(s_next);
            __syncthreads();  // everyone has read s_next before it is overwritten
        } else {
            t += gridDim.x;
        }
    }
}

__global__ void reset_counter(int* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

template <int BM, int BN, int WM, int WN>
hipError_t launch_shape(const GroupedLaunch& L, int grid, hipStream_t s) {
    const dim3 block(WM * WN * 64);
    const dim3 g(grid);
#define ROT_G(AK, BK, DYN) hipLaunchKernelGGL((grouped_f32_kernel<BM, BN, WM, WN, AK, BK, DYN>), g, block, 0, s, L)
    if (L.dynamic) {
        hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, s, L.counter);
        if (L.a_kcontig) {
            if (L.b_kcontig) ROT_G(true, true, true); else ROT_G(true, false, true);
        } else {
            if (L.b_kcontig) ROT_G(false, true, true); else ROT_G(false, false, true);
        }
    } else {
        if (L.a_kcontig) {
            if (L.b_kcontig) ROT_G(true, true, false); else ROT_G(true, false, false);
        } else {
            if (L.b_kcontig) ROT_G(false, true, false); else ROT_G(false, false, false);
        }
    }
#undef ROT_G
    return hipGetLastError();
}

}  // namespace

int grouped_tile_edge(GroupedShape shape) {
    switch (shape) {
        case GroupedShape::k128:
        case GroupedShape::k128d: return 128;
        case GroupedShape::k64: return 64;
        case GroupedShape::k32: return 32;
    }
    return 128;
}

hipError_t grouped_gemm_f32(const GroupedLaunch& L, hipStream_t stream) {
    if (L.n_tiles <= 0) return hipSuccess;
    if (L.dynamic && !L.counter) return hipErrorInvalidValue;
    const int grid = L.grid > 0 ? std::min(L.grid, L.n_tiles) : L.n_tiles;
    switch (L.shape) {
        case GroupedShape::k128: return launch_shape<128, 128, 2, 2>(L, grid, stream);
        case GroupedShape::k64: return launch_shape<64, 64, 2, 2>(L, grid, stream);
        case GroupedShape::k32: return launch_shape<32, 32, 1, 1>(L, grid, stream);
        case GroupedShape::k128d: {
            const dim3 g(grid), block(256);
#define ROT_GD(AK, BK, DYN) hipLaunchKernelGGL((grouped_f32_dl_kernel<AK, BK, DYN>), g, block, 0, stream, L)
            if (L.dynamic) {
                hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, stream, L.counter);
                if (L.a_kcontig) {
                    if (L.b_kcontig) ROT_GD(true, true, true); else ROT_GD(true, false, true);
                } else {
                    if (L.b_kcontig) ROT_GD(false, true, true); else ROT_GD(false, false, true);
                }
            } else {
                if (L.a_kcontig) {
                    if (L.b_kcontig) ROT_GD(true, true, false); else ROT_GD(true, false, false);
                } else {
                    if (L.b_kcontig) ROT_GD(false, true, false); else ROT_GD(false, false, false);
                }
            }
#undef ROT_GD
            return hipGetLastError();
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace rot
