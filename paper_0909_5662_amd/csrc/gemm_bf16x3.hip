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

__device__ inline int xcd_linear_id() {
    const int nwg = gridDim.x, wg = blockIdx.x;
    const int per = nwg / 8, rem = nwg % 8;
    const int xcd = wg % 8, idx = wg / 8;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

constexpr int kSlabK = 16;  // k per slab

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
constexpr int kBufferFlags = 0x00020000;
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
                                                                         int n_fastest) {
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
    } else {
        const int per_batch = tiles_m * tiles_n;
        bidx = lin / per_batch;
        const int rr = lin % per_batch;
        // neighbouring workgroups share the B panel (M tiles fastest) or the
        // A panel (N tiles fastest)
        m0 = (n_fastest ? rr / tiles_n : rr % tiles_m) * T;
        n0 = (n_fastest ? rr % tiles_n : rr / tiles_m) * T;
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
hipError_t launch_tile(const Bf16Desc& g, hipStream_t s) {
    constexpr int T = 32 * WGM * BI;
    const int tm = (g.M + T - 1) / T, tn = (g.N + T - 1) / T;
    if (g.upper && (EPI_T || g.M != g.N)) return hipErrorInvalidValue;
    const int64_t tiles = (g.upper ? (int64_t)tm * (tm + 1) / 2 : (int64_t)tm * tn) * g.batch;
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    const char* order = getenv("ROT_BF16_ORDER");
    const int nf = order ? (order[0] == 'n') : 0;
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

// 256 x 256 tiles (eight waves of 128 x 64, two per SIMD; a ring of 4 stages
// of 32 KB) when both output extents reach 256, else 128 x 128 (four waves
// of 64 x 64; 4 stages of 16 KB).  Environment ROT_BF16_CFG=128 forces the
// small tile and ROT_BF16_CFG=ring5 a ring of 5 stages (measurement knobs).
template <bool EPI_T>
hipError_t launch_bf16(const Bf16Desc& g, hipStream_t s) {
    const char* env = getenv("ROT_BF16_CFG");
    const bool small = env && !strcmp(env, "128");
    if (!small && g.M >= 256 && g.N >= 256) {
        if (env && !strcmp(env, "ring5")) return launch_tile<2, 4, 4, 2, 5, EPI_T>(g, s);
        return launch_tile<2, 4, 4, 2, 4, EPI_T>(g, s);
    }
    return launch_tile<2, 2, 2, 2, 4, EPI_T>(g, s);
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

// p has its leading dimensions resolved.
hipError_t rotate_bf16(const rot_problem& p, int b0, int nb, void* ws, bool symmetric, hipStream_t stream) {
    const Bf16Layout L = layout(p.m, p.d, p.mp);
    char* base = static_cast<char*>(ws);
    uint16_t* u1h = reinterpret_cast<uint16_t*>(base);
    uint16_t* u1l = reinterpret_cast<uint16_t*>(base + L.u1);
    uint16_t* u2h = reinterpret_cast<uint16_t*>(base + 2 * L.u1);
    uint16_t* u2l = reinterpret_cast<uint16_t*>(base + 2 * L.u1 + L.u2);
    uint16_t* th = reinterpret_cast<uint16_t*>(base + L.shared);
    uint16_t* tl = reinterpret_cast<uint16_t*>(base + L.shared + (size_t)nb * L.t_op);
    uint16_t* oh = reinterpret_cast<uint16_t*>(base + L.shared + 2 * (size_t)nb * L.t_op);
    uint16_t* ol = reinterpret_cast<uint16_t*>(base + L.shared + 2 * (size_t)nb * L.t_op + (size_t)nb * L.o_op);
    const int rows = p.m * p.d;
    if (b0 == 0) {
        const dim3 grid((p.mp + 63) / 64, (rows + 63) / 64);
        hipError_t e = prof_timed("split_u_bf16x3", stream, [&] {
            hipError_t err = zero_last_slab(u1h, u1l, L.u1_rows, p.m, 0, 1, stream);
            if (err == hipSuccess) err = zero_last_slab(u2h, u2l, L.u2_rows, rows, 0, 1, stream);
            if (err != hipSuccess) return err;
            hipLaunchKernelGGL(split_u_kernel, grid, dim3(256), 0, stream, static_cast<const float*>(p.U), rows,
                               p.mp, p.ldu, p.d, u1h, u1l, u2h, u2l);
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
    }
    // stage 1, transposed: C(beta*d+s, i) = sum_j U1(beta*d+s, j) O_b(i, j) = T_b(i, beta*d+s)
    Bf16Desc a{};
    a.M = p.d * p.mp;
    a.N = p.m;
    a.K = p.m;
    a.batch = nb;
    a.a_hi = u1h;
    a.a_lo = u1l;
    a.a_bs = 0;
    a.b_hi = oh;
    a.b_lo = ol;
    a.b_bs = (int64_t)(L.o_op / 2);
    a.t_hi = th;
    a.t_lo = tl;
    a.d = p.d;
    a.t_rows = p.mp;
    a.t_bs = (int64_t)(L.t_op / 2);
    hipError_t e = prof_timed("split_o_bf16x3", stream, [&] {
        // Tt's K padding (stage 1 writes only k < m*d); O's is written by the split
        hipError_t err = zero_last_slab(th, tl, p.mp, rows, (int64_t)(L.t_op / 2), nb, stream);
        if (err != hipSuccess) return err;
        const float* Ob = static_cast<const float*>(p.O) + (int64_t)b0 * p.stride_o;
        const dim3 grid((p.m + 63) / 64, (p.m + 63) / 64, nb);
        hipLaunchKernelGGL(split_o_kernel, grid, dim3(256), 0, stream, Ob, p.m, p.ldo, p.stride_o, oh, ol,
                           (int64_t)(L.o_op / 2));
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    e = prof_timed("stage1_bf16x3", stream, [&] { return launch_bf16<true>(a, stream); });
    if (e != hipSuccess) return e;
    // stage 2: out_b(alpha, beta) = sum_r U2(alpha, r) Tt_b(beta, r)
    Bf16Desc b{};
    b.M = p.mp;
    b.N = p.mp;
    b.K = p.m * p.d;
    b.batch = nb;
    b.a_hi = u2h;
    b.a_lo = u2l;
    b.a_bs = 0;
    b.b_hi = th;
    b.b_lo = tl;
    b.b_bs = (int64_t)(L.t_op / 2);
    b.c = static_cast<float*>(p.out) + (int64_t)b0 * p.stride_out;
    b.ldc = p.ldout;
    b.c_bs = p.stride_out;
    b.upper = symmetric ? 1 : 0;
    return prof_timed(symmetric ? "stage2sym_bf16x3" : "stage2_bf16x3", stream,
                      [&] { return launch_bf16<false>(b, stream); });
}

}  // namespace rot
