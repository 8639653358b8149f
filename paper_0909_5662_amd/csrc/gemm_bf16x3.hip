// Split-BF16 rotation: every FP32 operand x is carried as x = hi + lo with
// hi = bf16(x), lo = bf16(x - hi) (round to nearest even), and every product
// a*b as a_hi*b_hi + a_hi*b_lo + a_lo*b_hi on BF16 matrix cores with FP32
// accumulation (the dropped a_lo*b_lo term is below 2^-16 relative).
//
// BF16 matrix instructions take 8 consecutive k per lane, so both operands
// are kept K-contiguous:
//   stage 1  computed transposed, C = U1 O_b^T with C(beta*d+s, i) = T_b(i, beta*d+s):
//            A = U1[beta*d+s][j] = U[j*d+s][beta] (pre-split once per call),
//            B = O_b (pre-split by a streaming pass per chunk: splitting while
//            staging costs ~4 vector instructions per matrix instruction);
//            the epilogue splits C and stores it as Tt_b[beta][i*d+s], i.e. as
//            stage 2's B.
//   stage 2  out_b = U^T T_b :  A = U2[alpha][r] = U[r][alpha] (pre-split),
//            B = Tt_b; FP32 output.
// Stage 1's M index is ordered beta*d + s (site state fastest): the four
// consecutive rows of a lane's accumulator group are, for d = 4, the entries
// r = i*d + s, s < 4 of Tt[beta], one 8-byte store.
//
// Slab layout.  Every split operand (rows x K) is stored as K/16 slabs; slab
// q holds k = 16q..16q+15 of all rows, 32 bytes per row, row after row, and
// the two 16-byte halves of row r are swapped when bit 3 of r is set.  The
// 16-wide K slice of a tile is then one contiguous block per array, copied
// verbatim into LDS by buffer loads with LDS destination (1 KB per wave
// instruction, whole cache lines), and the swap spreads the 128-bit fragment
// reads of 16 lanes (rows c..c+15, one k half) over all 64 LDS banks.  The
// last slab of an operand whose K is not a multiple of 16 is zero beyond K.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "buffer_rsrc.h"
#include "lds_slice.h"
#include "rot_internal.h"

namespace rot {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 round to nearest even (the hardware conversion,
// v_cvt_pk_bf16_f32), as a bit pattern.
__device__ inline uint16_t rne_bf16(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ inline float bf16_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// hi/lo split of two values: {hi pair, lo pair}, each pair packed with the
// first value in the low half (one conversion instruction per pair).
__device__ inline u32x2 split2(float a, float b) {
    const bf16x2 h = {(__bf16)a, (__bf16)b};
    const bf16x2 l = {(__bf16)(a - (float)h[0]), (__bf16)(b - (float)h[1])};
    return u32x2{__builtin_bit_cast(uint32_t, h), __builtin_bit_cast(uint32_t, l)};
}


constexpr int kSlabK = 16;  // k per slab
constexpr int kDefaultOrder = 0;  // tile order of gemm_bf16x3_kernel (see launch_tile)

inline __host__ __device__ int64_t n_slabs(int64_t K) { return (K + kSlabK - 1) / kSlabK; }

// Element (r, k) of a slab-layout operand with `rows` rows.
inline __host__ __device__ int64_t slab_off(int64_t r, int64_t k, int64_t rows) {
    return (k >> 4) * rows * kSlabK + r * kSlabK + ((((k >> 3) & 1) ^ ((r >> 3) & 1)) << 3) + (k & 7);
}

struct Bf16Desc {
    int M, N, K, batch;
    // A: M rows, B: N rows, both K-contiguous slab layout, pre-split
    const uint16_t* a_hi;
    const uint16_t* a_lo;
    int64_t a_bs;
    const uint16_t* b_hi;
    const uint16_t* b_lo;
    int64_t b_bs;
    // plain epilogue: C[row*ldc + col] (FP32); with `upper` (M == N, symmetric
    // output) only tiles on or above the diagonal are computed and each
    // off-diagonal one is also stored transposed
    float* c;
    int64_t ldc, c_bs;
    int upper;
    // split-transposed epilogue: C(n = beta*d + s, i) -> T (t_rows rows,
    // slab layout), element (beta, i*d + s)
    uint16_t* t_hi;
    uint16_t* t_lo;
    int d;
    int64_t t_rows, t_bs;
};

// Buffer descriptor over one slab-layout operand (raw addressing; loads past
// its last slab return zero).
__device__ inline __amdgpu_buffer_rsrc_t operand_rsrc(const uint16_t* p, int rows, int K) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(p), (short)0,
                                             (int)(n_slabs(K) * rows * kSlabK * 2), kBufferFlags);
}

// s_waitcnt immediate that waits until at most n vector-memory operations
// of this wave are outstanding (other counters unconstrained).
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | 0x70 | 0xF00; }
// s_waitcnt immediate that waits for every LDS access of this wave.
constexpr int kLgkmcnt0 = 0xF | (3 << 14) | 0x70;

// Ordering point for the compiler only: memory accesses are not moved across
// it (s_barrier alone does not order them for the optimiser).
__device__ inline void compiler_fence() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }

// Write a wave's BI x BJ accumulator blocks (origin row0w, col0 of C):
// split-transposed into T (EPI_T) or plain FP32.  Accumulator element v of
// lane (h, c) of a 32 x 32 block is C(8*(v/4) + 4*h + v%4, c).
template <int BI, int BJ, bool EPI_T, bool D4>
__device__ inline void store_tile(const Bf16Desc& g, const f32x16 (&acc)[BI][BJ], int bidx, int row0w, int col0, int h,
                                  int c, bool mirror, bool diag) {
    if (EPI_T) {
        // C(n = beta*d + s, i) -> T(beta, i*d + s).  The four rows 4q..4q+3 a
        // lane holds in accumulator elements 4q..4q+3 are, for d = 4, the four
        // site states of one beta: k = 4i..4i+3, one 8-byte store per array.
        uint16_t* th = g.t_hi + (int64_t)bidx * g.t_bs;
        uint16_t* tl = g.t_lo + (int64_t)bidx * g.t_bs;
#pragma unroll
        for (int i = 0; i < BI; i++)
#pragma unroll
            for (int k = 0; k < BJ; k++) {
                const int col = col0 + k * 32 + c;  // old block state i
                if (col >= g.N) continue;
                const f32x16 a = acc[i][k];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const int row0 = row0w + i * 32 + 8 * q + 4 * h;
                    const u32x2 p0 = split2(a[4 * q], a[4 * q + 1]), p1 = split2(a[4 * q + 2], a[4 * q + 3]);
                    const u32x2 hv = {p0[0], p1[0]}, lv = {p0[1], p1[1]};
                    if (D4 && row0 + 4 <= g.M) {
                        const int64_t off = slab_off(row0 >> 2, (int64_t)col * 4, g.t_rows);
                        *reinterpret_cast<u32x2*>(th + off) = hv;
                        *reinterpret_cast<u32x2*>(tl + off) = lv;
                    } else if (!D4) {
#pragma unroll
                        for (int e = 0; e < 4; e++) {
                            const int row = row0 + e;
                            if (row < g.M) {
                                const int64_t off = slab_off(row / g.d, (int64_t)col * g.d + row % g.d, g.t_rows);
                                th[off] = (uint16_t)(hv[e >> 1] >> (16 * (e & 1)));
                                tl[off] = (uint16_t)(lv[e >> 1] >> (16 * (e & 1)));
                            }
                        }
                    }
                }
            }
    } else {
        float* cb = g.c + (int64_t)bidx * g.c_bs;
#pragma unroll
        for (int i = 0; i < BI; i++)
#pragma unroll
            for (int k = 0; k < BJ; k++) {
                const int col = col0 + k * 32 + c;
                if (col >= g.N) continue;
#pragma unroll
                for (int v = 0; v < 16; v++) {
                    const int row = row0w + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
                    // a diagonal tile of a symmetric output keeps row <= col and mirrors it
                    if (row < g.M && (!diag || row <= col)) {
                        cb[(int64_t)row * g.ldc + col] = acc[i][k][v];
                        if (diag && row < col) cb[(int64_t)col * g.ldc + row] = acc[i][k][v];
                    }
                }
            }
        if (mirror) {
            // the transposed tile: a lane's rows 8q + 4h .. +3 are four
            // consecutive entries of row `col`
            const bool vec4 = (g.ldc & 3) == 0 && (reinterpret_cast<uintptr_t>(cb) & 15) == 0;
#pragma unroll
            for (int i = 0; i < BI; i++)
#pragma unroll
                for (int k = 0; k < BJ; k++) {
                    const int col = col0 + k * 32 + c;
                    if (col >= g.N) continue;
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const int row0 = row0w + i * 32 + 8 * q + 4 * h;
                        float* p = cb + (int64_t)col * g.ldc + row0;
                        if (vec4 && row0 + 4 <= g.M) {
                            *reinterpret_cast<f32x4*>(p) = f32x4{acc[i][k][4 * q], acc[i][k][4 * q + 1],
                                                                 acc[i][k][4 * q + 2], acc[i][k][4 * q + 3]};
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; e++)
                                if (row0 + e < g.M) p[e] = acc[i][k][4 * q + e];
                        }
                    }
                }
        }
    }
}

// Square tile T x T as WGM x WGN waves of (32 BI) x (32 BJ), each BI x BJ
// blocks of v_mfma_f32_32x32x16_bf16.  That
// instruction takes from lane l A(row l%32, k 8*(l/32)+e) and B(k 8*(l/32)+e,
// col l%32), e < 8.  The K loop runs over slabs through a ring of S LDS
// stages, each holding one slab of A_hi, A_lo, B_hi, B_lo for the tile
// (T rows x 32 bytes per array, as in memory).  Vector memory fills the
// stages directly: wave w copies blocks w, w + waves, ... (32 rows, 1 KB
// each) of each array, one buffer load with LDS destination per block, 16
// bytes per lane.  S - 1 slabs are
// in flight while one is multiplied.  Before step t each wave waits for its
// own loads of slab t + 1, and the barrier makes every wave's loads visible
// and frees slab t - 1's stage (every wave consumed its fragments in step
// t - 1) for slab t + S - 1.  The fragments of slab t + 1 are read into a
// second register set while slab t is multiplied.
template <int WGM, int WGN, int BI, int BJ, int S, bool EPI_T, bool D4>
__global__ __launch_bounds__(64 * WGM * WGN, 1) void gemm_bf16x3_kernel(Bf16Desc g, int tiles_m, int tiles_n,
                                                                         int order) {
    constexpr int NW = WGM * WGN;
    constexpr int T = 32 * WGM * BI;
    static_assert(32 * WGN * BJ == T, "square tile");
    constexpr int NBLK = T / 32;     // 1 KB blocks per array in a stage
    static_assert(NBLK % NW == 0, "whole blocks per wave");
    constexpr int BPW = NBLK / NW;   // blocks per wave per array
    constexpr int ARR = T * kSlabK;  // elements of one array in a stage
    constexpr int STAGE = 4 * ARR;   // A_hi, A_lo, B_hi, B_lo
    constexpr int LOADS = 4 * BPW;   // direct loads per wave per stage
    __shared__ __attribute__((aligned(1024))) uint16_t lds[S * STAGE];

    const int lin = xcd_linear_id();
    int bidx, m0, n0;
    if (!EPI_T && g.upper) {
        // tiles (i, j), i <= j, column by column: r -> j(j+1)/2 + i
        const int per_batch = tiles_m * (tiles_m + 1) / 2;
        bidx = lin / per_batch;
        const int r = lin % per_batch;
        int j = (int)((sqrtf(8.0f * (float)r + 1.0f) - 1.0f) * 0.5f);
        while (j * (j + 1) / 2 > r) j--;
        while ((j + 1) * (j + 2) / 2 <= r) j++;
        m0 = (r - j * (j + 1) / 2) * T;
        n0 = j * T;
    } else if (order > 0) {
        // grouped order: the columns of every batch element side by side
        // (column = bidx * tiles_n + n tile); workgroups sweep them in groups
        // of `order` M tiles, M tiles fastest, so a run of consecutive
        // workgroups (which run together on one XCD) shares `order` A panels
        // and about run/order B panels
        const int cols = tiles_n * (int)(gridDim.x / (tiles_m * tiles_n));
        const int per_group = order * cols;
        const int grp = lin / per_group, first = grp * order;
        const int gsize = min(tiles_m - first, order);
        const int r = lin % per_group;
        m0 = (first + r % gsize) * T;
        const int col = r / gsize;
        bidx = col / tiles_n;
        n0 = (col % tiles_n) * T;
    } else {
        const int per_batch = tiles_m * tiles_n;
        bidx = lin / per_batch;
        const int rr = lin % per_batch;
        // neighbouring workgroups share the B panel (M tiles fastest) or the
        // A panel (N tiles fastest, order < 0)
        m0 = (order < 0 ? rr / tiles_n : rr % tiles_m) * T;
        n0 = (order < 0 ? rr % tiles_n : rr / tiles_m) * T;
    }

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    const int h = lane >> 5, c = lane & 31;

    const __amdgpu_buffer_rsrc_t rs[4] = {operand_rsrc(g.a_hi + (int64_t)bidx * g.a_bs, g.M, g.K),
                                          operand_rsrc(g.a_lo + (int64_t)bidx * g.a_bs, g.M, g.K),
                                          operand_rsrc(g.b_hi + (int64_t)bidx * g.b_bs, g.N, g.K),
                                          operand_rsrc(g.b_lo + (int64_t)bidx * g.b_bs, g.N, g.K)};
    // byte offsets of this lane's 16 bytes in slab 0, and the slab strides
    const uint32_t a_off = (uint32_t)((m0 + wave * 32) * kSlabK * 2 + lane * 16);
    const uint32_t b_off = (uint32_t)((n0 + wave * 32) * kSlabK * 2 + lane * 16);
    const uint32_t a_slab = (uint32_t)g.M * kSlabK * 2, b_slab = (uint32_t)g.N * kSlabK * 2;
    const int nk = (int)n_slabs(g.K);

    // wave w copies blocks w, w + NW, ... (32 rows each) of every array
    auto issue = [&](int st) {
        uint16_t* base = lds + (st % S) * STAGE + wave * 512;
#pragma unroll
        for (int j = 0; j < 4; j++)
#pragma unroll
            for (int x = 0; x < BPW; x++)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rs[j], (__attribute__((address_space(3))) void*)(base + j * ARR + x * NW * 512), 16,
                    (j < 2 ? a_off + (uint32_t)st * a_slab : b_off + (uint32_t)st * b_slab) +
                        (uint32_t)(x * NW * 1024),
                    0, 0, 0);
    };

    f32x16 acc[BI][BJ];
#pragma unroll
    for (int i = 0; i < BI; i++)
#pragma unroll
        for (int j = 0; j < BJ; j++)
#pragma unroll
            for (int v = 0; v < 16; v++) acc[i][j][v] = 0.f;

    // fragment slot of this lane: rows c (+ multiples of 32) and k half h
    const int fslot = (h ^ ((c >> 3) & 1)) * 8;
    struct Frags {
        bf16x8 ah[BI], al[BI], bh[BJ], bl[BJ];
    };
    auto read = [&](Frags& f, int st) {
        const uint16_t* sb = lds + (st % S) * STAGE;
#pragma unroll
        for (int i = 0; i < BI; i++) {
            const int ra = (wm * 32 * BI + i * 32 + c) * kSlabK + fslot;
            f.ah[i] = *reinterpret_cast<const bf16x8*>(sb + ra);
            f.al[i] = *reinterpret_cast<const bf16x8*>(sb + ARR + ra);
        }
#pragma unroll
        for (int j = 0; j < BJ; j++) {
            const int rb = (wn * 32 * BJ + j * 32 + c) * kSlabK + fslot;
            f.bh[j] = *reinterpret_cast<const bf16x8*>(sb + 2 * ARR + rb);
            f.bl[j] = *reinterpret_cast<const bf16x8*>(sb + 3 * ARR + rb);
        }
    };
    auto multiply = [&](const Frags& f) {
        // small terms first; consecutive instructions use different accumulators
#pragma unroll
        for (int i = 0; i < BI; i++)
#pragma unroll
            for (int k = 0; k < BJ; k++)
                acc[i][k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.al[i], f.bh[k], acc[i][k], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < BI; i++)
#pragma unroll
            for (int k = 0; k < BJ; k++)
                acc[i][k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.ah[i], f.bl[k], acc[i][k], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < BI; i++)
#pragma unroll
            for (int k = 0; k < BJ; k++)
                acc[i][k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.ah[i], f.bh[k], acc[i][k], 0, 0, 0);
    };
    // wait until this wave's loads of slab `st` are done, given that slabs up
    // to min(st + later, nk - 1) have been issued; then the barrier
    auto wait_stage = [&](int st, int later) {
        if (st + later < nk) {
            if (later == S - 2)
                __builtin_amdgcn_s_waitcnt(vmcnt_imm(LOADS * (S - 2)));
            else
                __builtin_amdgcn_s_waitcnt(vmcnt_imm(LOADS * (S - 3)));
        } else {
            __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
        }
        compiler_fence();
        __builtin_amdgcn_s_barrier();
        compiler_fence();
    };

    for (int st = 0; st < S - 1 && st < nk; st++) issue(st);
    Frags f0, f1;
    wait_stage(0, S - 2);
    read(f0, 0);
    auto step = [&](int t, Frags& cur, Frags& nxt) {
        // the reads of `cur` (issued a step ago) complete before the reads of
        // `nxt` start, so the matrix instructions below wait for nothing
        __builtin_amdgcn_s_waitcnt(kLgkmcnt0);
        if (t + 1 < nk) {
            wait_stage(t + 1, S - 3);
            if (t + S - 1 < nk) issue(t + S - 1);
        }
        // the next slab's fragments (on the last step a finished stage is
        // read and not used), interleaved with this slab's products so the
        // waves' LDS reads spread over the matrix work instead of arriving
        // together after the barrier
        read(nxt, t + 1);
        multiply(cur);
#pragma unroll
        for (int i = 0; i < 2 * (BI + BJ); i++) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
            __builtin_amdgcn_sched_group_barrier(0x008, (3 * BI * BJ) / (2 * (BI + BJ)), 0);  // matrix instructions
        }
        compiler_fence();
    };
    for (int t = 0; t < nk; t += 2) {
        step(t, f0, f1);
        if (t + 1 < nk) step(t + 1, f1, f0);
    }
    store_tile<BI, BJ, EPI_T, D4>(g, acc, bidx, m0 + wm * 32 * BI, n0 + wn * 32 * BJ, h, c,
                                  !EPI_T && g.upper && m0 != n0, !EPI_T && g.upper && m0 == n0);
}

// Variant with the B fragments loaded straight from global memory into
// registers: in the slab layout a fragment (32 rows x one 16-byte k half) is
// 1 KB of contiguous bytes, one buffer load per array.  Only A goes through
// the LDS ring (S stages of A_hi, A_lo), so LDS carries half the copy writes
// and two thirds of the fragment reads of gemm_bf16x3_kernel.  The prologue
// issues A slabs 0 .. S-2 and B slabs 0, 1; every step t then issues A slab
// t + S - 1 (direct to LDS) and B slab t + 2 (to one of three register
// sets), past the last slab too (those loads read beyond the operand and
// return zeros, into stages and sets no longer used), so each wait counts a
// known number of later loads (smaller in the first steps).  The A
// fragments of slab t + 1 are read from LDS row block by row block, each
// right after the products of slab t that used the same registers.  Per
// accumulator the products come in the same order as in gemm_bf16x3_kernel,
// so the two kernels give the same bits.
template <int WGM, int WGN, int BI, int BJ, int S, bool EPI_T, bool D4>
__global__ __launch_bounds__(64 * WGM * WGN, 1) void gemm_bf16x3_db_kernel(Bf16Desc g, int tiles_m, int tiles_n,
                                                                            int order) {
    constexpr int NW = WGM * WGN;
    constexpr int T = 32 * WGM * BI;
    static_assert(32 * WGN * BJ == T, "square tile");
    constexpr int NBLK = T / 32;     // 1 KB blocks per array in a stage
    static_assert(NBLK % NW == 0, "whole blocks per wave");
    constexpr int BPW = NBLK / NW;   // blocks per wave per array
    constexpr int ARR = T * kSlabK;  // elements of one array in a stage
    constexpr int STAGE = 2 * ARR;   // A_hi, A_lo
    constexpr int LA = 2 * BPW;      // direct loads per wave per step
    constexpr int LB = 2 * BJ;       // B fragment loads per wave per step
    static_assert(S >= 3, "ring depth");
    // loads issued after the one waited for: slab 0's A before the first
    // step; slab t + 1's A at step t (t < S - 3 in the prologue's order,
    // otherwise one step's B and S - 3 whole steps); slab t's B at step t
    constexpr int WAIT_A0 = (S - 2) * LA + 2 * LB;
    constexpr int WAIT_A = (S - 3) * LA + (S - 2) * LB;
    constexpr int WAIT_B = 2 * (LA + LB), WAIT_B0 = LA + 2 * LB;
    static_assert(S >= 4 && S <= 6 && WAIT_A0 <= 63 && WAIT_A <= 63 && WAIT_B <= 63, "vmcnt range");
    __shared__ __attribute__((aligned(1024))) uint16_t lds[S * STAGE];

    const int lin = xcd_linear_id();
    int bidx, m0, n0;
    if (order > 0) {
        const int cols = tiles_n * (int)(gridDim.x / (tiles_m * tiles_n));
        const int per_group = order * cols;
        const int grp = lin / per_group, first = grp * order;
        const int gsize = min(tiles_m - first, order);
        const int r = lin % per_group;
        m0 = (first + r % gsize) * T;
        const int col = r / gsize;
        bidx = col / tiles_n;
        n0 = (col % tiles_n) * T;
    } else {
        const int per_batch = tiles_m * tiles_n;
        bidx = lin / per_batch;
        const int rr = lin % per_batch;
        m0 = (order < 0 ? rr / tiles_n : rr % tiles_m) * T;
        n0 = (order < 0 ? rr % tiles_n : rr / tiles_m) * T;
    }

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    const int h = lane >> 5, c = lane & 31;

    const __amdgpu_buffer_rsrc_t ra[2] = {operand_rsrc(g.a_hi + (int64_t)bidx * g.a_bs, g.M, g.K),
                                          operand_rsrc(g.a_lo + (int64_t)bidx * g.a_bs, g.M, g.K)};
    const __amdgpu_buffer_rsrc_t rb[2] = {operand_rsrc(g.b_hi + (int64_t)bidx * g.b_bs, g.N, g.K),
                                          operand_rsrc(g.b_lo + (int64_t)bidx * g.b_bs, g.N, g.K)};
    const uint32_t a_off = (uint32_t)((m0 + wave * 32) * kSlabK * 2 + lane * 16);
    const uint32_t a_slab = (uint32_t)g.M * kSlabK * 2, b_slab = (uint32_t)g.N * kSlabK * 2;
    const int nk = (int)n_slabs(g.K);
    // fragment slot of this lane: rows c (+ multiples of 32) and k half h
    const int fslot = (h ^ ((c >> 3) & 1)) * 8;
    // byte offset of this lane's B fragment of block j in slab 0
    const uint32_t b_off = (uint32_t)(((n0 + wn * 32 * BJ + c) * kSlabK + fslot) * 2);

    auto issue_a = [&](int st) __attribute__((always_inline)) {
        uint16_t* base = lds + (st % S) * STAGE + wave * 512;
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int x = 0; x < BPW; x++)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    ra[j], (__attribute__((address_space(3))) void*)(base + j * ARR + x * NW * 512), 16,
                    a_off + (uint32_t)st * a_slab + (uint32_t)(x * NW * 1024), 0, 0, 0);
    };
    struct BSet {
        bf16x8 bh[BJ], bl[BJ];
    };
    // slab st's B fragments (a negative or past-the-end slab reads zeros)
    auto issue_b = [&](BSet& o, int st) __attribute__((always_inline)) {
        const uint32_t off = b_off + (uint32_t)st * b_slab;
#pragma unroll
        for (int j = 0; j < BJ; j++) {
            o.bh[j] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rb[0], off + j * 1024, 0, 0));
            o.bl[j] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rb[1], off + j * 1024, 0, 0));
        }
    };

    f32x16 acc[BI][BJ];
#pragma unroll
    for (int i = 0; i < BI; i++)
#pragma unroll
        for (int j = 0; j < BJ; j++)
#pragma unroll
            for (int v = 0; v < 16; v++) acc[i][j][v] = 0.f;

    bf16x8 ah[BI], al[BI];
    auto read_a = [&](int i, int st) __attribute__((always_inline)) {
        const uint16_t* sb = lds + (st % S) * STAGE;
        const int ra_ = (wm * 32 * BI + i * 32 + c) * kSlabK + fslot;
        ah[i] = *reinterpret_cast<const bf16x8*>(sb + ra_);
        al[i] = *reinterpret_cast<const bf16x8*>(sb + ARR + ra_);
    };
    auto barrier = [&]() __attribute__((always_inline)) {
        compiler_fence();
        __builtin_amdgcn_s_barrier();
        compiler_fence();
    };

    // the wait counts assume exactly this issue order: fences keep the
    // compiler from reordering the loads
    BSet bs[3];
#pragma unroll
    for (int st = 0; st <= S - 2; st++) {
        issue_a(st);
        compiler_fence();
    }
    issue_b(bs[0], 0);
    compiler_fence();
    issue_b(bs[1], 1);
    compiler_fence();
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(WAIT_A0));
    barrier();
#pragma unroll
    for (int i = 0; i < BI; i++) read_a(i, 0);

    // Step t on B set CUR, filling set NB with slab t + 2; WA, WB: the
    // immediate waits for slab t + 1's A and slab t's B.  A macro, so that the
    // counts stay compile-time immediates and the steady loop has no branches
    // (the compiler's own waits are then no stricter than these).
#define BF16_DB_STEP(T_, CUR, NB, WA, WB)                                                                \
    do {                                                                                                  \
        const int t_ = (T_);                                                                              \
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(WA));                                                        \
        barrier();                                                                                        \
        issue_a(t_ + S - 1);                                                                              \
        compiler_fence();                                                                                 \
        issue_b(NB, t_ + 2);                                                                              \
        compiler_fence();                                                                                 \
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(WB));                                                        \
        compiler_fence();                                                                                 \
        _Pragma("unroll") for (int i = 0; i < BI; i++) {                                                  \
            _Pragma("unroll") for (int k = 0; k < BJ; k++) acc[i][k] =                                    \
                __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], (CUR).bh[k], acc[i][k], 0, 0, 0);          \
            _Pragma("unroll") for (int k = 0; k < BJ; k++) acc[i][k] =                                    \
                __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], (CUR).bl[k], acc[i][k], 0, 0, 0);          \
            _Pragma("unroll") for (int k = 0; k < BJ; k++) acc[i][k] =                                    \
                __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], (CUR).bh[k], acc[i][k], 0, 0, 0);          \
            read_a(i, t_ + 1);                                                                            \
        }                                                                                                 \
        compiler_fence();                                                                                 \
    } while (0)
    // later loads when slab t + 1's A is waited for in the first steps (the
    // prologue's order), then in every later step
    constexpr int WA0 = (S - 3) * LA + 2 * LB;
    constexpr int WA1 = S >= 5 ? (S - 3) * LA + 3 * LB : WAIT_A;
    constexpr int WA2 = S >= 6 ? (S - 3) * LA + 4 * LB : WAIT_A;
    // slab t uses set t % 3 and fills set (t + 2) % 3; the first three steps
    // (nk >= 3 is required) run outside the loop so that the loop begins in
    // the state its back edge leaves
    BF16_DB_STEP(0, bs[0], bs[2], WA0, WAIT_B0);
    BF16_DB_STEP(1, bs[1], bs[0], WA1, WAIT_B);
    BF16_DB_STEP(2, bs[2], bs[1], WA2, WAIT_B);
    int t = 3;
    for (; t + 3 <= nk; t += 3) {
        BF16_DB_STEP(t, bs[0], bs[2], WAIT_A, WAIT_B);
        BF16_DB_STEP(t + 1, bs[1], bs[0], WAIT_A, WAIT_B);
        BF16_DB_STEP(t + 2, bs[2], bs[1], WAIT_A, WAIT_B);
    }
    // the last one or two steps wait for every earlier load: their own B
    // loads are never used, and the compiler may drop them, which would
    // shorten the counts above
    if (t < nk) BF16_DB_STEP(t, bs[0], bs[2], 0, 0);
    if (t + 1 < nk) BF16_DB_STEP(t + 1, bs[1], bs[0], 0, 0);
#undef BF16_DB_STEP
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    __builtin_amdgcn_s_waitcnt(kLgkmcnt0);
    store_tile<BI, BJ, EPI_T, D4>(g, acc, bidx, m0 + wm * 32 * BI, n0 + wn * 32 * BJ, h, c, false, false);
}

// U (rows = m*d, cols = mp, row stride ldu), row r = j*d + s, both split
// into hi/lo (slab layout):
//   U1 (d*mp rows, K = m):   element (beta*d + s, j) = U[j*d+s][beta]
//   U2 (mp rows, K = m*d):   element (alpha, r)      = U[r][alpha]
// 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void split_u_kernel(const float* __restrict__ U, int rows, int cols, int64_t ldu,
                                                      int d, uint16_t* __restrict__ u1h, uint16_t* __restrict__ u1l,
                                                      uint16_t* __restrict__ u2h, uint16_t* __restrict__ u2l) {
    __shared__ float tile[64][65];
    const int r0 = blockIdx.y * 64, a0 = blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const int r = r0 + ty + 4 * k, a = a0 + tx;
        tile[ty + 4 * k][tx] = (r < rows && a < cols) ? U[(int64_t)r * ldu + a] : 0.f;
    }
    __syncthreads();
    const int r = r0 + tx;
    if (r >= rows) return;
    const int j = r / d, s = r % d;
    const int64_t rows1 = (int64_t)d * cols;
#pragma unroll 4
    for (int k = 0; k < 16; k++) {
        const int a = a0 + ty + 4 * k;
        if (a >= cols) break;
        const float x = tile[tx][ty + 4 * k];
        const uint16_t hh = rne_bf16(x);
        const uint16_t ll = rne_bf16(x - bf16_f32(hh));
        const int64_t o2 = slab_off(a, r, cols);
        u2h[o2] = hh;
        u2l[o2] = ll;
        const int64_t o1 = slab_off((int64_t)a * d + s, j, rows1);
        u1h[o1] = hh;
        u1l[o1] = ll;
    }
}

// O_b (m x m at O + b*stride_o, row stride ldo) -> hi/lo at b*ob in slab
// layout (m rows, K = m), one 64 x 64 block per workgroup.  Rows are read into LDS (16-byte
// loads when the block lies inside O and its rows are 16-byte aligned), then
// each thread converts 8 values (one k half of one row in one slab) and
// writes them as one 16-byte chunk per array.  Each 16 lanes take 16
// consecutive rows and the same k half, so with a row pitch of 68 floats
// both the 16-byte LDS writes and reads touch all 64 banks once.  Columns
// past m in the last slab are written as zero.
__global__ __launch_bounds__(256) void split_o_kernel(const float* __restrict__ O, int m, int64_t ldo,
                                                      int64_t stride_o, uint16_t* __restrict__ oh,
                                                      uint16_t* __restrict__ ol, int64_t ob) {
    __shared__ __attribute__((aligned(16))) float tile[64][68];
    const int b = blockIdx.z, i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const float* src = O + (int64_t)b * stride_o;
    const int tid = threadIdx.x;
    if (j0 + 64 <= m && (ldo & 3) == 0 && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int r = (tid >> 4) + 16 * k, c4 = (tid & 15) * 4, i = i0 + r;
            f32x4 v = {0.f, 0.f, 0.f, 0.f};
            if (i < m) v = *reinterpret_cast<const f32x4*>(src + (int64_t)i * ldo + j0 + c4);
            *reinterpret_cast<f32x4*>(&tile[r][c4]) = v;
        }
    } else {
        const int tx = tid & 63, ty = tid >> 6;
#pragma unroll
        for (int k = 0; k < 16; k++) {
            const int i = i0 + ty + 4 * k, j = j0 + tx;
            tile[ty + 4 * k][tx] = (i < m && j < m) ? src[(int64_t)i * ldo + j] : 0.f;
        }
    }
    __syncthreads();
    uint16_t* dh = oh + (int64_t)b * ob;
    uint16_t* dl = ol + (int64_t)b * ob;
    const int64_t nslab = n_slabs(m);
#pragma unroll
    for (int x = 0; x < 2; x++) {
        const int ch = tid + 256 * x;  // slab q, k half, row
        const int q = ch >> 7, half = (ch >> 6) & 1, row = ch & 63;
        const int i = i0 + row;
        const int64_t sq = j0 / kSlabK + q;  // global slab index
        if (i >= m || sq >= nslab) continue;
        const f32x4 v0 = *reinterpret_cast<const f32x4*>(&tile[row][q * kSlabK + half * 8]);
        const f32x4 v1 = *reinterpret_cast<const f32x4*>(&tile[row][q * kSlabK + half * 8 + 4]);
        const u32x2 p0 = split2(v0[0], v0[1]), p1 = split2(v0[2], v0[3]);
        const u32x2 p2 = split2(v1[0], v1[1]), p3 = split2(v1[2], v1[3]);
        const u32x4 hv = {p0[0], p1[0], p2[0], p3[0]}, lv = {p0[1], p1[1], p2[1], p3[1]};
        const int slot = half ^ ((i >> 3) & 1);  // slab layout: halves swapped when bit 3 of the row is set
        const int64_t off = sq * (int64_t)m * kSlabK + (int64_t)i * kSlabK + slot * 8;
        *reinterpret_cast<u32x4*>(dh + off) = hv;
        *reinterpret_cast<u32x4*>(dl + off) = lv;
    }
}

// `len` elements at a + b*bstride and at l + b*bstride, b < gridDim.y, set
// to zero.
__global__ __launch_bounds__(256) void zero_pair_kernel(uint16_t* __restrict__ a, uint16_t* __restrict__ l,
                                                        int64_t len, int64_t bstride) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= len) return;
    const int64_t off = (int64_t)blockIdx.y * bstride + i;
    a[off] = 0;
    l[off] = 0;
}

// Zero the K padding of `batch` slab-layout operands (rows x K, bstride
// elements apart): their whole last slab when K is not a multiple of 16,
// before the producer writes its valid part.
hipError_t zero_last_slab(uint16_t* a, uint16_t* l, int64_t rows, int64_t K, int64_t bstride, int batch,
                          hipStream_t s) {
    if (K % kSlabK == 0 || rows <= 0 || batch <= 0) return hipSuccess;
    const int64_t len = rows * kSlabK, off = (n_slabs(K) - 1) * len;
    hipLaunchKernelGGL(zero_pair_kernel, dim3((unsigned)((len + 255) / 256), (unsigned)batch), dim3(256), 0, s,
                       a + off, l + off, len, bstride);
    return hipGetLastError();
}

template <int WGM, int WGN, int BI, int BJ, int S, bool EPI_T>
hipError_t launch_tile(const Bf16Desc& g, int nf, hipStream_t s) {
    constexpr int T = 32 * WGM * BI;
    const int tm = (g.M + T - 1) / T, tn = (g.N + T - 1) / T;
    if (g.upper && (EPI_T || g.M != g.N)) return hipErrorInvalidValue;
    const int64_t tiles = (g.upper ? (int64_t)tm * (tm + 1) / 2 : (int64_t)tm * tn) * g.batch;
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    // with d = 4 the row extent d*mp is a multiple of 4, so every group of
    // four rows is complete and the vector store path covers all of them
    if (EPI_T && g.d == 4)
        hipLaunchKernelGGL((gemm_bf16x3_kernel<WGM, WGN, BI, BJ, S, EPI_T, true>), dim3((unsigned)tiles),
                           dim3(64 * WGM * WGN), 0, s, g, tm, tn, nf);
    else
        hipLaunchKernelGGL((gemm_bf16x3_kernel<WGM, WGN, BI, BJ, S, EPI_T, false>), dim3((unsigned)tiles),
                           dim3(64 * WGM * WGN), 0, s, g, tm, tn, nf);
    return hipGetLastError();
}

// A launch configuration: tile edge (256: eight waves of 128 x 64, two per
// SIMD, ring stages of 32 KB; 128: four waves of 64 x 64, stages of 16 KB),
// ring depth (4 or 5 stages) and tile order (0: M tiles fastest per batch
// element; -1: N tiles fastest; G > 0: groups of G M tiles across all
// columns).  256 applies only when both output extents reach 256.
// (Bf16Cfg and Bf16Choice are declared in rot_internal.h.)

// The environment's measurement knobs override a configuration:
// ROT_BF16_CFG=128 | ring5 | direct5 | direct6, ROT_BF16_ORDER=m | n | G.
Bf16Cfg with_env(Bf16Cfg c) {
    const char* env = getenv("ROT_BF16_CFG");
    if (env && !strcmp(env, "128")) c.tile = 128;
    if (env && !strcmp(env, "ring5")) c.ring = 5;
    if (env && !strncmp(env, "direct", 6)) {
        c.tile = 256;
        c.direct = 1;
        c.ring = env[6] == '6' ? 6 : 5;
    }
    const char* ord = getenv("ROT_BF16_ORDER");
    if (ord) c.order = ord[0] == 'n' ? -1 : ord[0] == 'm' ? 0 : std::max(0, atoi(ord));
    return c;
}

template <int WGM, int WGN, int BI, int BJ, int S, bool EPI_T>
hipError_t launch_tile_db(const Bf16Desc& g, int nf, hipStream_t s) {
    constexpr int T = 32 * WGM * BI;
    const int tm = (g.M + T - 1) / T, tn = (g.N + T - 1) / T;
    const int64_t tiles = (int64_t)tm * tn * g.batch;
    if (g.upper || tiles > 0x7fffffff) return hipErrorInvalidValue;
    if (EPI_T && g.d == 4)
        hipLaunchKernelGGL((gemm_bf16x3_db_kernel<WGM, WGN, BI, BJ, S, EPI_T, true>), dim3((unsigned)tiles),
                           dim3(64 * WGM * WGN), 0, s, g, tm, tn, nf);
    else
        hipLaunchKernelGGL((gemm_bf16x3_db_kernel<WGM, WGN, BI, BJ, S, EPI_T, false>), dim3((unsigned)tiles),
                           dim3(64 * WGM * WGN), 0, s, g, tm, tn, nf);
    return hipGetLastError();
}

template <bool EPI_T>
hipError_t launch_bf16(const Bf16Desc& g, const Bf16Cfg& cfg0, hipStream_t s) {
    const Bf16Cfg cfg = with_env(cfg0);
    if (cfg.direct && cfg.tile == 256 && g.M >= 256 && g.N >= 256 && !g.upper && n_slabs(g.K) >= 3) {
        if (cfg.ring == 6) return launch_tile_db<2, 4, 4, 2, 6, EPI_T>(g, cfg.order, s);
        return launch_tile_db<2, 4, 4, 2, 5, EPI_T>(g, cfg.order, s);
    }
    if (cfg.tile == 256 && g.M >= 256 && g.N >= 256) {
        if (cfg.ring == 5) return launch_tile<2, 4, 4, 2, 5, EPI_T>(g, cfg.order, s);
        return launch_tile<2, 4, 4, 2, 4, EPI_T>(g, cfg.order, s);
    }
    return launch_tile<2, 2, 2, 2, 4, EPI_T>(g, cfg.order, s);
}

template <bool EPI_T>
hipError_t launch_bf16(const Bf16Desc& g, hipStream_t s) {
    return launch_bf16<EPI_T>(g, Bf16Cfg{}, s);
}

struct Bf16Layout {
    int64_t u1_rows, u2_rows;  // rows of U1 (d*mp) and U2 (mp)
    size_t u1, u2, t_op;       // bytes of one hi (or lo) array
    size_t o_op;               // bytes of one operator's split O (hi or lo)
    size_t shared;             // bytes of the pre-split U (4 arrays)
};

inline size_t al256(size_t n) { return (n + 255) / 256 * 256; }

Bf16Layout layout(int m, int d, int mp) {
    Bf16Layout L;
    L.u1_rows = (int64_t)d * mp;
    L.u2_rows = mp;
    L.u1 = al256((size_t)(n_slabs(m) * L.u1_rows * kSlabK * 2));
    L.u2 = al256((size_t)(n_slabs((int64_t)m * d) * mp * kSlabK * 2));
    L.t_op = L.u2;  // Tt_b: mp rows, K = m*d
    L.o_op = al256((size_t)(n_slabs(m) * m * kSlabK * 2));
    L.shared = 2 * L.u1 + 2 * L.u2;
    return L;
}

// X (R x C FP32 per batch element, row stride ldx, batch stride bsx; with
// SYM, R == C and the values are X + X^T) split into hi/lo slab layouts:
//   rows layout (R rows, K = C): element (r, c) -> rh/rl + b*rbs
//   cols layout (C rows, K = R): element (c, r) -> ch/cl + b*cbs
// Either pair may be null.  The K padding of each layout's last slab is
// written as zero, so operands concatenated along K (one slab array after
// the other) multiply to exact zeros there.  One 64 x 64 tile per workgroup
// through LDS (with SYM also the mirror tile); each thread then converts 8
// consecutive k of one row of a layout and stores them as one 16-byte chunk
// per array.
template <bool SYM>
__global__ __launch_bounds__(256) void split_layouts_kernel(const float* __restrict__ X, int R, int C, int64_t ldx,
                                                            int64_t bsx, uint16_t* __restrict__ rh,
                                                            uint16_t* __restrict__ rl, int64_t rbs,
                                                            uint16_t* __restrict__ ch, uint16_t* __restrict__ cl,
                                                            int64_t cbs) {
    __shared__ float tile[64][65];
    __shared__ float mir[SYM ? 64 : 1][65];
    const int b = blockIdx.z, r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    const float* src = X + (int64_t)b * bsx;
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const int r = r0 + ty + 4 * k, c = c0 + tx;
        tile[ty + 4 * k][tx] = (r < R && c < C) ? src[(int64_t)r * ldx + c] : 0.f;
        if (SYM) {
            // mir[i][j] = X(c0 + i, r0 + j): rows of the mirror block, coalesced
            const int mr = c0 + ty + 4 * k, mc = r0 + tx;
            mir[ty + 4 * k][tx] = (mr < C && mc < R) ? src[(int64_t)mr * ldx + mc] : 0.f;
        }
    }
    __syncthreads();
    auto value = [&](int i, int j) {  // element (r0 + i, c0 + j)
        return SYM ? tile[i][j] + mir[j][i] : tile[i][j];
    };
    auto store8 = [&](uint16_t* hi, uint16_t* lo, int64_t off, const float (&v)[8]) {
        const u32x2 p0 = split2(v[0], v[1]), p1 = split2(v[2], v[3]);
        const u32x2 p2 = split2(v[4], v[5]), p3 = split2(v[6], v[7]);
        *reinterpret_cast<u32x4*>(hi + off) = u32x4{p0[0], p1[0], p2[0], p3[0]};
        *reinterpret_cast<u32x4*>(lo + off) = u32x4{p0[1], p1[1], p2[1], p3[1]};
    };
    if (rh) {
        const int kpad = (int)(n_slabs(C) * kSlabK);
#pragma unroll
        for (int x = 0; x < 2; x++) {
            const int q = tid + 256 * x, i = q & 63, k8 = (q >> 6) * 8;
            const int r = r0 + i, k0 = c0 + k8;
            if (r >= R || k0 >= kpad) continue;
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; e++) v[e] = value(i, k8 + e);
            store8(rh + (int64_t)b * rbs, rl + (int64_t)b * rbs, slab_off(r, k0, R), v);
        }
    }
    if (ch) {
        const int kpad = (int)(n_slabs(R) * kSlabK);
#pragma unroll
        for (int x = 0; x < 2; x++) {
            const int q = tid + 256 * x, j = q & 63, k8 = (q >> 6) * 8;
            const int c = c0 + j, k0 = r0 + k8;
            if (c >= C || k0 >= kpad) continue;
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; e++) v[e] = value(k8 + e, j);
            store8(ch + (int64_t)b * cbs, cl + (int64_t)b * cbs, slab_off(c, k0, C), v);
        }
    }
}

// Enqueue split_layouts_kernel over `batch` matrices.
hipError_t split_layouts(const float* X, int R, int C, int64_t ldx, int64_t bsx, int batch, bool sym, uint16_t* rh,
                         uint16_t* rl, int64_t rbs, uint16_t* ch, uint16_t* cl, int64_t cbs, hipStream_t s) {
    if (R <= 0 || C <= 0 || batch <= 0) return hipSuccess;
    const dim3 grid((unsigned)((C + 63) / 64), (unsigned)((R + 63) / 64), (unsigned)batch);
    if (sym)
        hipLaunchKernelGGL(split_layouts_kernel<true>, grid, dim3(256), 0, s, X, R, C, ldx, bsx, rh, rl, rbs, ch, cl,
                           cbs);
    else
        hipLaunchKernelGGL(split_layouts_kernel<false>, grid, dim3(256), 0, s, X, R, C, ldx, bsx, rh, rl, rbs, ch,
                           cl, cbs);
    return hipGetLastError();
}

}  // namespace

// Every split operand array, with one tile (256 rows) of overhang, must stay
// below 2 GiB: loads address it with 32-bit byte offsets.
bool bf16_shape_supported(int m, int d, int mp) {
    const Bf16Layout L = layout(m, d, mp);
    const size_t lim = (size_t)1 << 31, over = 256 * kSlabK * 2;
    return L.u1 + over < lim && L.u2 + over < lim && L.o_op + over < lim;
}

size_t bf16_group_workspace(int m, int d, int mp, int ops) {
    const Bf16Layout L = layout(m, d, mp);
    return L.shared + (size_t)ops * 2 * (L.t_op + L.o_op);
}

namespace {

// Pointers into the split-BF16 workspace for a chunk of nb operators.
struct Bf16Ws {
    uint16_t *u1h, *u1l, *u2h, *u2l, *th, *tl, *oh, *ol;
};

Bf16Ws carve(const Bf16Layout& L, void* ws, int nb) {
    char* base = static_cast<char*>(ws);
    Bf16Ws w;
    w.u1h = reinterpret_cast<uint16_t*>(base);
    w.u1l = reinterpret_cast<uint16_t*>(base + L.u1);
    w.u2h = reinterpret_cast<uint16_t*>(base + 2 * L.u1);
    w.u2l = reinterpret_cast<uint16_t*>(base + 2 * L.u1 + L.u2);
    w.th = reinterpret_cast<uint16_t*>(base + L.shared);
    w.tl = reinterpret_cast<uint16_t*>(base + L.shared + (size_t)nb * L.t_op);
    w.oh = reinterpret_cast<uint16_t*>(base + L.shared + 2 * (size_t)nb * L.t_op);
    w.ol = reinterpret_cast<uint16_t*>(base + L.shared + 2 * (size_t)nb * L.t_op + (size_t)nb * L.o_op);
    return w;
}

// U split once per call (b0 == 0), then the chunk's O split and the K
// padding of its Tt.
hipError_t split_inputs(const rot_problem& p, const Bf16Layout& L, const Bf16Ws& w, int b0, int nb,
                        hipStream_t stream) {
    const int rows = p.m * p.d;
    if (b0 == 0) {
        const dim3 grid((p.mp + 63) / 64, (rows + 63) / 64);
        hipError_t e = prof_timed("split_u_bf16x3", stream, [&] {
            hipError_t err = zero_last_slab(w.u1h, w.u1l, L.u1_rows, p.m, 0, 1, stream);
            if (err == hipSuccess) err = zero_last_slab(w.u2h, w.u2l, L.u2_rows, rows, 0, 1, stream);
            if (err != hipSuccess) return err;
            hipLaunchKernelGGL(split_u_kernel, grid, dim3(256), 0, stream, static_cast<const float*>(p.U), rows,
                               p.mp, p.ldu, p.d, w.u1h, w.u1l, w.u2h, w.u2l);
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
    }
    return prof_timed("split_o_bf16x3", stream, [&] {
        // Tt's K padding (stage 1 writes only k < m*d); O's is written by the split
        hipError_t err = zero_last_slab(w.th, w.tl, p.mp, rows, (int64_t)(L.t_op / 2), nb, stream);
        if (err != hipSuccess) return err;
        const float* Ob = static_cast<const float*>(p.O) + (int64_t)b0 * p.stride_o;
        const dim3 grid((p.m + 63) / 64, (p.m + 63) / 64, nb);
        hipLaunchKernelGGL(split_o_kernel, grid, dim3(256), 0, stream, Ob, p.m, p.ldo, p.stride_o, w.oh, w.ol,
                           (int64_t)(L.o_op / 2));
        return hipGetLastError();
    });
}

// stage 1, transposed: C(beta*d+s, i) = sum_j U1(beta*d+s, j) O_b(i, j) = T_b(i, beta*d+s)
Bf16Desc stage1_desc(const rot_problem& p, const Bf16Layout& L, const Bf16Ws& w, int nb) {
    Bf16Desc a{};
    a.M = p.d * p.mp;
    a.N = p.m;
    a.K = p.m;
    a.batch = nb;
    a.a_hi = w.u1h;
    a.a_lo = w.u1l;
    a.a_bs = 0;
    a.b_hi = w.oh;
    a.b_lo = w.ol;
    a.b_bs = (int64_t)(L.o_op / 2);
    a.t_hi = w.th;
    a.t_lo = w.tl;
    a.d = p.d;
    a.t_rows = p.mp;
    a.t_bs = (int64_t)(L.t_op / 2);
    return a;
}

// stage 2: out_b(alpha, beta) = sum_r U2(alpha, r) Tt_b(beta, r)
Bf16Desc stage2_desc(const rot_problem& p, const Bf16Layout& L, const Bf16Ws& w, int b0, int nb, bool symmetric) {
    Bf16Desc b{};
    b.M = p.mp;
    b.N = p.mp;
    b.K = p.m * p.d;
    b.batch = nb;
    b.a_hi = w.u2h;
    b.a_lo = w.u2l;
    b.a_bs = 0;
    b.b_hi = w.th;
    b.b_lo = w.tl;
    b.b_bs = (int64_t)(L.t_op / 2);
    b.c = static_cast<float*>(p.out) + (int64_t)b0 * p.stride_out;
    b.ldc = p.ldout;
    b.c_bs = p.stride_out;
    b.upper = symmetric ? 1 : 0;
    return b;
}

const Bf16Cfg kCandidates[] = {{256, 4, kDefaultOrder, 0}, {256, 5, kDefaultOrder, 0}, {128, 4, kDefaultOrder, 0},
                               {256, 5, kDefaultOrder, 1}, {256, 6, kDefaultOrder, 1}};

std::string cfg_token(const Bf16Cfg& c) {
    return std::to_string(c.tile) + (c.direct ? "d" : "r") + std::to_string(c.ring);
}

bool parse_cfg(const std::string& t, Bf16Cfg* c) {
    for (const Bf16Cfg& k : kCandidates)
        if (t == cfg_token(k)) {
            *c = k;
            return true;
        }
    return false;
}

// Device name and compute-unit count of the current device, for tuning keys.
std::string device_tag() {
    int dev = 0, n_cu = 0;
    hipDeviceProp_t props;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess ||
        hipGetDeviceProperties(&props, dev) != hipSuccess)
        return "unknown";
    std::string arch = props.gcnArchName;
    return arch.substr(0, arch.find(':')) + "|cu" + std::to_string(n_cu);
}

// Milliseconds of `launch` on `stream` (one warm-up run, then the mean of two).
float time_ms(hipStream_t stream, const std::function<hipError_t()>& launch, hipError_t* err) {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(a, stream);
    for (int r = 0; r < 2 && e == hipSuccess; r++) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 1e30f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    *err = e;
    return ms / 2;
}

}  // namespace

// The launch configurations of the two stages for this shape: from the tuning
// cache, else (when `may_tune` and no measurement knob is set) by timing
// every candidate on the first chunk of nb operators (its results are
// overwritten by the call that follows), else the defaults.  Every
// configuration gives the same bits: each output element sums the same
// products slab by slab in the same order, whatever the tile.
hipError_t bf16_choice(const rot_problem& p, int nb, bool symmetric, void* ws, bool may_tune, hipStream_t stream,
                       Bf16Choice* choice) {
    *choice = Bf16Choice{};
    const std::string key = "bf16|" + device_tag() + "|m" + std::to_string(p.m) + "|d" + std::to_string(p.d) +
                            "|mp" + std::to_string(p.mp) + "|nb" + std::to_string(nb) + (symmetric ? "|sym" : "");
    std::vector<std::string> t;
    if (tune_get(key, &t) && t.size() == 2 && parse_cfg(t[0], &choice->s1) && parse_cfg(t[1], &choice->s2))
        return hipSuccess;
    const char* off = getenv("ROT_AUTOTUNE");
    if (!may_tune || (off && !strcmp(off, "0")) || getenv("ROT_BF16_CFG") || getenv("ROT_BF16_ORDER"))
        return hipSuccess;
    const Bf16Layout L = layout(p.m, p.d, p.mp);
    const Bf16Ws w = carve(L, ws, nb);
    const Bf16Desc a = stage1_desc(p, L, w, nb), b = stage2_desc(p, L, w, 0, nb, symmetric);
    // below 256 in both extents of both stages only the 128 tile applies
    if ((a.M < 256 || a.N < 256) && (b.M < 256 || b.N < 256)) return hipSuccess;
    hipError_t e = split_inputs(p, L, w, 0, nb, stream);
    if (e != hipSuccess) return e;
    float best1 = 1e30f, best2 = 1e30f;
    for (const Bf16Cfg& c : kCandidates) {
        if (c.tile == 256 && !(a.M >= 256 && a.N >= 256)) continue;
        const float ms = time_ms(stream, [&] { return launch_bf16<true>(a, c, stream); }, &e);
        if (e != hipSuccess) return e;
        if (ms < best1) {
            best1 = ms;
            choice->s1 = c;
        }
    }
    for (const Bf16Cfg& c : kCandidates) {
        if (c.tile == 256 && !(b.M >= 256 && b.N >= 256)) continue;
        const float ms = time_ms(stream, [&] { return launch_bf16<false>(b, c, stream); }, &e);
        if (e != hipSuccess) return e;
        if (ms < best2) {
            best2 = ms;
            choice->s2 = c;
        }
    }
    log_msg(2, "%s: stage 1 %s (%.3f ms), stage 2 %s (%.3f ms)", key.c_str(), cfg_token(choice->s1).c_str(), best1,
            cfg_token(choice->s2).c_str(), best2);
    tune_put(key, {cfg_token(choice->s1), cfg_token(choice->s2)});
    return hipSuccess;
}

// p has its leading dimensions resolved.
hipError_t rotate_bf16(const rot_problem& p, int b0, int nb, void* ws, bool symmetric, const Bf16Choice& choice,
                       hipStream_t stream) {
    const Bf16Layout L = layout(p.m, p.d, p.mp);
    const Bf16Ws w = carve(L, ws, nb);
    hipError_t e = split_inputs(p, L, w, b0, nb, stream);
    if (e != hipSuccess) return e;
    const Bf16Desc a = stage1_desc(p, L, w, nb);
    e = prof_timed("stage1_bf16x3", stream, [&] { return launch_bf16<true>(a, choice.s1, stream); });
    if (e != hipSuccess) return e;
    const Bf16Desc b = stage2_desc(p, L, w, b0, nb, symmetric);
    return prof_timed(symmetric ? "stage2sym_bf16x3" : "stage2_bf16x3", stream,
                      [&] { return launch_bf16<false>(b, choice.s2, stream); });
}


// ---------------------------------------------------------------------------
// Split-BF16 adjoint.  With P_b = U dOut_b and Q_b = U dOut_b^T ((m*d) x mp,
// viewed as m x d*mp through the row index i*d + s):
//   dO_b = P_b,r U_r^T
//   dU_r = sum_b O_b^T P_b,r + O_b Q_b,r    (symmetric O_b: sum_b O_b (P_b + Q_b)_r)
// Every product is a split-BF16 GEMM (three BF16 products per operand pair,
// FP32 accumulation) whose operands are FP32 values split into the slab
// layout: U and U_r once per call, dOut_b (transposed; rows for Q, or
// dOut_b + dOut_b^T for the symmetric sum), P/Q (rows and transposed
// layouts) and O_b per operator chunk.  The dU operator sum is one GEMM
// whose K runs over (operator, i) of every term, cut into parts whose
// partial sums are added in a fixed order.
// ---------------------------------------------------------------------------
namespace {

struct Bf16Bwd {
    int64_t mK;          // m rounded up to a whole slab
    size_t ua, ur;       // one hi or lo array: U (m*d rows, K = mp), U_r (m rows, K = d*mp)
    size_t dq;           // dOut_b in one layout (mp rows, K = mp)
    size_t p32;          // P_b or Q_b in FP32 ((m*d) x mp)
    size_t pa;           // P_b,r rows layout (m rows, K = d*mp)
    size_t pb;           // P_b,r / Q_b,r transposed layout (d*mp rows, K = m)
    size_t os;           // O_b (or O_b^T) (m rows, K = m)
    size_t part;         // a partial dU (FP32, (m*d) x mp)
    size_t shared() const { return 2 * ua + 2 * ur; }
    size_t per_op() const { return 4 * dq + p32 + 2 * pa + 4 * pb + 4 * os; }
};

Bf16Bwd bwd_layout(int m, int d, int mp) {
    Bf16Bwd L;
    const int64_t md = (int64_t)m * d, dmp = (int64_t)d * mp;
    L.mK = n_slabs(m) * kSlabK;
    L.ua = al256((size_t)(n_slabs(mp) * md * kSlabK * 2));
    L.ur = al256((size_t)(n_slabs(dmp) * m * kSlabK * 2));
    L.dq = al256((size_t)(n_slabs(mp) * mp * kSlabK * 2));
    L.p32 = al256((size_t)md * mp * 4);
    L.pa = L.ur;
    // arrays concatenated along K must follow each other with no gap: their
    // sizes are whole slabs of whole rows (multiples of 32 bytes), not rounded
    L.pb = (size_t)(n_slabs(m) * dmp * kSlabK * 2);
    L.os = (size_t)(n_slabs(m) * m * kSlabK * 2);
    L.part = al256((size_t)md * mp * 4);
    return L;
}

constexpr size_t kOperandLimit = ((size_t)1 << 31) - 256 * kSlabK * 2;  // 32-bit byte offsets

// Parts of the dU sum over `terms` (operator, factor) terms: enough output
// tiles to fill the chip, at most 8, and each part's operands below 2 GiB.
int bwd_parts(const Bf16Bwd& L, int m, int d, int mp, int terms) {
    const int64_t dmp = (int64_t)d * mp;
    const int T = (m >= 256 && dmp >= 256) ? 256 : 128;
    const int64_t tiles = ((m + T - 1) / T) * ((dmp + T - 1) / T);
    int parts = (int)std::min<int64_t>(8, (1024 + tiles - 1) / tiles);
    const size_t biggest = std::max(L.pb, L.os);
    const int per_part_max = (int)std::max<size_t>(1, kOperandLimit / biggest);
    parts = std::max(parts, (terms + per_part_max - 1) / per_part_max);
    return std::max(1, std::min(parts, terms));
}

Bf16Desc plain_desc(int M, int N, int K, int batch, const uint16_t* ah, const uint16_t* al, int64_t abs_,
                    const uint16_t* bh, const uint16_t* bl, int64_t bbs, float* c, int64_t ldc, int64_t cbs) {
    Bf16Desc g{};
    g.M = M; g.N = N; g.K = K; g.batch = batch;
    g.a_hi = ah; g.a_lo = al; g.a_bs = abs_;
    g.b_hi = bh; g.b_lo = bl; g.b_bs = bbs;
    g.c = c; g.ldc = ldc; g.c_bs = cbs;
    return g;
}

}  // namespace

bool bf16_backward_supported(int m, int d, int mp) {
    const Bf16Bwd L = bwd_layout(m, d, mp);
    return L.ua < kOperandLimit && L.ur < kOperandLimit && L.pb < kOperandLimit && L.dq < kOperandLimit &&
           L.os < kOperandLimit;
}

// Workspace for `ops` operators per chunk (general operators: both dU terms).
size_t bf16_backward_workspace(int m, int d, int mp, int ops) {
    const Bf16Bwd L = bwd_layout(m, d, mp);
    // the four concatenated operand regions are each rounded up to 256 bytes
    return L.shared() + (size_t)ops * L.per_op() + 4 * 256 + (size_t)bwd_parts(L, m, d, mp, 2 * ops) * L.part;
}

// One chunk of nb operators from b0 (p resolved, U packed to row stride mp).
// dOut_b at dout + (b0 + b)*sd (sd = 0: one matrix for all).  dO/dU may be
// null.  dU accumulates when b0 > 0.
hipError_t backward_bf16(const rot_problem& p, int b0, int nb, const float* dout, int64_t sd, float* dO, float* dU,
                         bool sym, void* ws, hipStream_t s) {
    const Bf16Bwd L = bwd_layout(p.m, p.d, p.mp);
    const int m = p.m, d = p.d, mp = p.mp;
    const int md = m * d, dmp = d * mp;
    char* base = static_cast<char*>(ws);
    auto take = [&](size_t bytes) {
        uint16_t* q = reinterpret_cast<uint16_t*>(base);
        base += bytes;
        return q;
    };
    uint16_t *uah = take(L.ua), *ual = take(L.ua), *urh = take(L.ur), *url = take(L.ur);
    uint16_t *dth = take(nb * L.dq), *dtl = take(nb * L.dq), *dsh = take(nb * L.dq), *dsl = take(nb * L.dq);
    float* P = reinterpret_cast<float*>(take(nb * L.p32));
    uint16_t *pah = take(nb * L.pa), *pal = take(nb * L.pa);
    uint16_t *pbh = take(al256(2 * nb * L.pb)), *pbl = take(al256(2 * nb * L.pb));
    uint16_t *osh = take(al256(2 * nb * L.os)), *osl = take(al256(2 * nb * L.os));
    float* part = reinterpret_cast<float*>(base);
    const float* U = static_cast<const float*>(p.U);
    const int64_t e_dq = (int64_t)(L.dq / 2), e_pa = (int64_t)(L.pa / 2), e_pb = (int64_t)(L.pb / 2),
                  e_os = (int64_t)(L.os / 2), e_p32 = (int64_t)(L.p32 / 4);
    const int nd = sd == 0 ? 1 : nb;  // distinct upstream gradients in this chunk
    const int64_t bd = sd == 0 ? 0 : e_dq;
    hipError_t e = hipSuccess;
    if (b0 == 0) {
        // U (m*d rows, K = mp) and U_r (m rows, K = d*mp), both row layouts
        e = prof_timed("adj_split_u_bf16x3", s, [&] {
            hipError_t err = split_layouts(U, md, mp, mp, 0, 1, false, uah, ual, 0, nullptr, nullptr, 0, s);
            if (err == hipSuccess)
                err = split_layouts(U, m, dmp, dmp, 0, 1, false, urh, url, 0, nullptr, nullptr, 0, s);
            return err;
        });
        if (e != hipSuccess) return e;
    }
    const float* g0 = dout + (int64_t)b0 * sd;
    // dOut_b transposed (B of P = U dOut_b), and for dU the B of the second
    // term: dOut_b itself (Q = U dOut_b^T) or dOut_b + dOut_b^T (symmetric O)
    e = prof_timed("adj_split_dout_bf16x3", s, [&] {
        hipError_t err = split_layouts(g0, mp, mp, mp, sd, nd, false, nullptr, nullptr, 0, dth, dtl, e_dq, s);
        if (err == hipSuccess && dU)
            err = split_layouts(g0, mp, mp, mp, sd, nd, sym, dsh, dsl, e_dq, nullptr, nullptr, 0, s);
        return err;
    });
    if (e != hipSuccess) return e;
    const bool need_p = dO || (dU && !sym);
    if (need_p) {
        // P_b = U dOut_b (FP32), then P_b,r in the layouts its products read
        e = prof_timed("adj_P_bf16x3", s, [&] {
            return launch_bf16<false>(plain_desc(md, mp, mp, nb, uah, ual, 0, dth, dtl, bd, P, mp, e_p32), s);
        });
        if (e == hipSuccess)
            e = prof_timed("adj_split_p_bf16x3", s, [&] {
                return split_layouts(P, m, dmp, dmp, e_p32, nb, false, dO ? pah : nullptr, pal, e_pa,
                                     (dU && !sym) ? pbh : nullptr, pbl, e_pb, s);
            });
        if (e != hipSuccess) return e;
    }
    if (dO) {
        e = prof_timed("adj_dO_bf16x3", s, [&] {
            return launch_bf16<false>(plain_desc(m, m, dmp, nb, pah, pal, e_pa, urh, url, 0,
                                                 dO + (int64_t)b0 * m * m, m, (int64_t)m * m), s);
        });
        if (e != hipSuccess) return e;
    }
    if (!dU) return hipSuccess;
    // second term: Q_b = U dOut_b^T, or (P + Q)_b for symmetric operators,
    // transposed P_r layout after the first term's (general) or alone
    const int64_t qoff = sym ? 0 : (int64_t)nb * e_pb;
    e = prof_timed(sym ? "adj_PQ_bf16x3" : "adj_Q_bf16x3", s, [&] {
        return launch_bf16<false>(plain_desc(md, mp, mp, nb, uah, ual, 0, dsh, dsl, bd, P, mp, e_p32), s);
    });
    if (e == hipSuccess)
        e = prof_timed("adj_split_p_bf16x3", s, [&] {
            return split_layouts(P, m, dmp, dmp, e_p32, nb, false, nullptr, nullptr, 0, pbh + qoff, pbl + qoff,
                                 e_pb, s);
        });
    // A operands: O_b^T for the first term, O_b for the second (rows j, K i)
    if (e == hipSuccess)
        e = prof_timed("adj_split_o_bf16x3", s, [&] {
            const float* O = static_cast<const float*>(p.O) + (int64_t)b0 * p.stride_o;
            const int64_t ooff = sym ? 0 : (int64_t)nb * e_os;
            return split_layouts(O, m, m, p.ldo, p.stride_o, nb, false, osh + ooff, osl + ooff, e_os,
                                 sym ? nullptr : osh, osl, e_os, s);
        });
    if (e != hipSuccess) return e;
    // dU_r = sum over the terms t of A_t (m x mK) B_t^T (d*mp rows, K = mK),
    // K concatenated over terms and cut into np parts of q or q + 1 terms
    const int terms = sym ? nb : 2 * nb;
    const int np = bwd_parts(L, m, d, mp, terms);
    const int q = terms / np, r = terms % np;
    const int64_t mK = L.mK;
    e = prof_timed("adj_dU_bf16x3", s, [&] {
        hipError_t err = hipSuccess;
        if (r > 0)
            err = launch_bf16<false>(plain_desc(m, dmp, (int)((q + 1) * mK), r, osh, osl, (q + 1) * e_os, pbh, pbl,
                                                (q + 1) * e_pb, part, dmp, e_p32), s);
        if (err == hipSuccess) {
            const int64_t t0 = (int64_t)r * (q + 1);
            err = launch_bf16<false>(plain_desc(m, dmp, (int)(q * mK), np - r, osh + t0 * e_os, osl + t0 * e_os,
                                                q * e_os, pbh + t0 * e_pb, pbl + t0 * e_pb, q * e_pb,
                                                part + (int64_t)r * e_p32, dmp, e_p32), s);
        }
        return err;
    });
    if (e != hipSuccess) return e;
    return prof_timed("adj_dU_sum", s, [&] {
        return sum_parts(dU, part, (int64_t)md * mp, np, e_p32, b0 > 0, false, s);
    });
}

}  // namespace rot
