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
// Tiles are 256 x 256 (four waves of 128 x 128) so that each 128-bit LDS
// fragment read feeds 3 x 4 matrix instructions.
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
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;
constexpr int kSlice = 16;   // K elements per LDS slice: one matrix step
constexpr int kPitch = 24;   // LDS row pitch in bf16 elements (48 bytes): conflict-free 128-bit reads

__device__ inline uint16_t rne_bf16(float x) {
    const uint32_t b = __float_as_uint(x);
    if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu)) return (uint16_t)((b >> 16) | 0x40u);
    return (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline int xcd_linear_id() {
    const int nwg = gridDim.x, wg = blockIdx.x;
    const int per = nwg / 8, rem = nwg % 8;
    const int xcd = wg % 8, idx = wg / 8;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

struct Bf16Desc {
    int M, N, K, batch;
    // A (M x K, K-contiguous), pre-split
    const uint16_t* a_hi;
    const uint16_t* a_lo;
    int64_t lda, a_bs;
    // B (N x K, K-contiguous), pre-split
    const uint16_t* b_hi;
    const uint16_t* b_lo;
    int64_t ldb, b_bs;
    // plain epilogue: C[row*ldc + col] (FP32)
    float* c;
    int64_t ldc, c_bs;
    // split-transposed epilogue: C(n = beta*d + s, i) -> T[beta*t_ld + i*d + s]
    uint16_t* t_hi;
    uint16_t* t_lo;
    int d;
    int64_t t_ld, t_bs;
};

// Stage an R x KS slice of a pre-split K-contiguous operand into LDS with
// row pitch KS + 8: 2 arrays x R rows x KS/8 chunks of 16 bytes.
template <int R, int KS = kSlice>
struct SplitSlice {
    static constexpr int CPR = KS / 8;                 // chunks per row
    static constexpr int CH = 2 * R * CPR / kThreads;  // chunks per thread
    static constexpr int PITCH = KS + 8;
    u16x8 r[CH];
    __device__ inline void load(const uint16_t* __restrict__ hi, const uint16_t* __restrict__ lo, int64_t ld,
                                int r0, int rows, int k0, int ks, int tid) {
        if (r0 + R <= rows && k0 + KS <= ks) {  // interior slice: unconditional vector loads
#pragma unroll
            for (int c = 0; c < CH; c++) {
                const int f = tid + c * kThreads;
                const int arr = f / (CPR * R), q = f % (CPR * R);
                r[c] = *reinterpret_cast<const u16x8*>((arr ? lo : hi) + (int64_t)(r0 + q / CPR) * ld + k0 +
                                                       (q % CPR) * 8);
            }
            return;
        }
#pragma unroll
        for (int c = 0; c < CH; c++) {
            const int f = tid + c * kThreads;
            const int arr = f / (CPR * R), q = f % (CPR * R);
            const int row = q / CPR, k = (q % CPR) * 8;
            const int gr = r0 + row, gk = k0 + k;
            const uint16_t* p = (arr ? lo : hi) + (int64_t)gr * ld + gk;
#pragma unroll
            for (int e = 0; e < 8; e++) r[c][e] = (gr < rows && gk + e < ks) ? p[e] : (uint16_t)0;
        }
    }
    __device__ inline void store(uint16_t* s_hi, uint16_t* s_lo, int tid) const {
#pragma unroll
        for (int c = 0; c < CH; c++) {
            const int f = tid + c * kThreads;
            const int arr = f / (CPR * R), q = f % (CPR * R);
            *reinterpret_cast<u16x8*>((arr ? s_lo : s_hi) + (q / CPR) * PITCH + (q % CPR) * 8) = r[c];
        }
    }
};

// Tile BM x BN = (2*BI*32) x (2*BJ*32): four waves in a 2 x 2 grid, each
// BI x BJ blocks of v_mfma_f32_32x32x16_bf16.  That instruction takes from
// lane l A(row l%32, k 8*(l/32)+e) and B(k 8*(l/32)+e, col l%32), e < 8, and
// leaves C(8*(v/4) + 4*(l/32) + v%4, l%32) in accumulator element v.  An LDS
// slice holds KS values of k (KS/16 matrix steps); with the row pitch KS + 8
// (48 or 80 bytes) the 128-bit fragment reads of 16 lanes hit 16 distinct
// 4-bank groups.  Slice t+1 is fetched from HBM while slice t is multiplied.
template <int BI, int BJ, int KS, bool EPI_T, bool D4>
__global__ __launch_bounds__(kThreads, 1) void gemm_bf16x3_kernel(Bf16Desc g, int tiles_m, int tiles_n,
                                                                  int n_fastest) {
    constexpr int BM = 64 * BI, BN = 64 * BJ;
    constexpr int PITCH = KS + 8;
    constexpr int A_ARR = BM * PITCH, B_ARR = BN * PITCH;
    constexpr int BUF = 2 * A_ARR + 2 * B_ARR;
    __shared__ __attribute__((aligned(16))) uint16_t lds[2 * BUF];  // per buffer: A_hi, A_lo, B_hi, B_lo

    const int lin = xcd_linear_id();
    const int per_batch = tiles_m * tiles_n;
    const int bidx = lin / per_batch;
    const int rr = lin % per_batch;
    // neighbouring workgroups share the B panel (M tiles fastest) or the A
    // panel (N tiles fastest)
    const int m0 = (n_fastest ? rr / tiles_n : rr % tiles_m) * BM;
    const int n0 = (n_fastest ? rr % tiles_n : rr / tiles_m) * BN;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int h = lane >> 5, c = lane & 31;

    SplitSlice<BM, KS> la;
    SplitSlice<BN, KS> lb;
    const uint16_t* ah_g = g.a_hi + (int64_t)bidx * g.a_bs;
    const uint16_t* al_g = g.a_lo + (int64_t)bidx * g.a_bs;
    const uint16_t* bh_g = g.b_hi + (int64_t)bidx * g.b_bs;
    const uint16_t* bl_g = g.b_lo + (int64_t)bidx * g.b_bs;
    const int nk = (g.K + KS - 1) / KS;

    f32x16 acc[BI][BJ];
#pragma unroll
    for (int i = 0; i < BI; i++)
#pragma unroll
        for (int j = 0; j < BJ; j++)
#pragma unroll
            for (int v = 0; v < 16; v++) acc[i][j][v] = 0.f;

    auto A_hi = [&](int b) { return lds + b * BUF; };
    auto A_lo = [&](int b) { return lds + b * BUF + A_ARR; };
    auto B_hi = [&](int b) { return lds + b * BUF + 2 * A_ARR; };
    auto B_lo = [&](int b) { return lds + b * BUF + 2 * A_ARR + B_ARR; };

    la.load(ah_g, al_g, g.lda, m0, g.M, 0, g.K, tid);
    lb.load(bh_g, bl_g, g.ldb, n0, g.N, 0, g.K, tid);
    la.store(A_hi(0), A_lo(0), tid);
    lb.store(B_hi(0), B_lo(0), tid);
    __syncthreads();

    for (int t = 0; t < nk; t++) {
        const int cur = t & 1;
        if (t + 1 < nk) {
            la.load(ah_g, al_g, g.lda, m0, g.M, (t + 1) * KS, g.K, tid);
            lb.load(bh_g, bl_g, g.ldb, n0, g.N, (t + 1) * KS, g.K, tid);
        }
#pragma unroll
        for (int ks = 0; ks < KS / 16; ks++) {
            bf16x8 ah[BI], al[BI], bhv[BJ], blv[BJ];
#pragma unroll
            for (int i = 0; i < BI; i++) {
                const int ra = (wm * 32 * BI + i * 32 + c) * PITCH + ks * 16 + h * 8;
                ah[i] = *reinterpret_cast<const bf16x8*>(A_hi(cur) + ra);
                al[i] = *reinterpret_cast<const bf16x8*>(A_lo(cur) + ra);
            }
#pragma unroll
            for (int j = 0; j < BJ; j++) {
                const int rb = (wn * 32 * BJ + j * 32 + c) * PITCH + ks * 16 + h * 8;
                bhv[j] = *reinterpret_cast<const bf16x8*>(B_hi(cur) + rb);
                blv[j] = *reinterpret_cast<const bf16x8*>(B_lo(cur) + rb);
            }
            // small terms first; consecutive instructions use different accumulators
#pragma unroll
            for (int i = 0; i < BI; i++)
#pragma unroll
                for (int k = 0; k < BJ; k++)
                    acc[i][k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bhv[k], acc[i][k], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < BI; i++)
#pragma unroll
                for (int k = 0; k < BJ; k++)
                    acc[i][k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], blv[k], acc[i][k], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < BI; i++)
#pragma unroll
                for (int k = 0; k < BJ; k++)
                    acc[i][k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bhv[k], acc[i][k], 0, 0, 0);
        }
        if (t + 1 < nk) {
            la.store(A_hi(cur ^ 1), A_lo(cur ^ 1), tid);
            lb.store(B_hi(cur ^ 1), B_lo(cur ^ 1), tid);
        }
        __syncthreads();
    }

    if (EPI_T) {
        // C(n = beta*d + s, i) -> T[beta][i*d + s].  The four rows 4q..4q+3 a
        // lane holds in accumulator elements 4q..4q+3 are, for d = 4, the four
        // site states of one beta: one 8-byte store per array.
        uint16_t* th = g.t_hi + (int64_t)bidx * g.t_bs;
        uint16_t* tl = g.t_lo + (int64_t)bidx * g.t_bs;
#pragma unroll
        for (int i = 0; i < BI; i++)
#pragma unroll
            for (int k = 0; k < BJ; k++) {
                const int col = n0 + wn * 32 * BJ + k * 32 + c;  // old block state i
                if (col >= g.N) continue;
                const f32x16 a = acc[i][k];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const int row0 = m0 + wm * 32 * BI + i * 32 + 8 * q + 4 * h;
                    u16x4 hv, lv;
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        const float x = a[4 * q + e];
                        hv[e] = rne_bf16(x);
                        lv[e] = rne_bf16(x - bf16_f32(hv[e]));
                    }
                    if (D4 && row0 + 4 <= g.M) {
                        const int64_t off = (int64_t)(row0 >> 2) * g.t_ld + (int64_t)col * 4;
                        *reinterpret_cast<u16x4*>(th + off) = hv;
                        *reinterpret_cast<u16x4*>(tl + off) = lv;
                    } else if (!D4) {
#pragma unroll
                        for (int e = 0; e < 4; e++) {
                            const int row = row0 + e;
                            if (row < g.M) {
                                const int64_t off = (int64_t)(row / g.d) * g.t_ld + (int64_t)col * g.d + row % g.d;
                                th[off] = hv[e];
                                tl[off] = lv[e];
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
                const int col = n0 + wn * 32 * BJ + k * 32 + c;
                if (col >= g.N) continue;
#pragma unroll
                for (int v = 0; v < 16; v++) {
                    const int row = m0 + wm * 32 * BI + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
                    if (row < g.M) cb[(int64_t)row * g.ldc + col] = acc[i][k][v];
                }
            }
    }
}

// U (rows = m*d, cols = mp) -> U1[(beta*d+s)*ld1 + j] = U[j*d+s][beta]  (ld1 >= m)
//                            U2[alpha*ld2 + r]     = U[r][alpha]        (ld2 >= m*d)
// both split into hi/lo.  64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void split_u_kernel(const float* __restrict__ U, int rows, int cols, int d,
                                                      uint16_t* __restrict__ u1h, uint16_t* __restrict__ u1l,
                                                      int64_t ld1, uint16_t* __restrict__ u2h,
                                                      uint16_t* __restrict__ u2l, int64_t ld2) {
    __shared__ float tile[64][65];
    const int r0 = blockIdx.y * 64, a0 = blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const int r = r0 + ty + 4 * k, a = a0 + tx;
        tile[ty + 4 * k][tx] = (r < rows && a < cols) ? U[(int64_t)r * cols + a] : 0.f;
    }
    __syncthreads();
    const int r = r0 + tx;
    if (r >= rows) return;
    const int j = r / d, s = r % d;
#pragma unroll 4
    for (int k = 0; k < 16; k++) {
        const int a = a0 + ty + 4 * k;
        if (a >= cols) break;
        const float x = tile[tx][ty + 4 * k];
        const uint16_t hh = rne_bf16(x);
        const uint16_t ll = rne_bf16(x - bf16_f32(hh));
        u2h[(int64_t)a * ld2 + r] = hh;
        u2l[(int64_t)a * ld2 + r] = ll;
        const int64_t o1 = ((int64_t)a * d + s) * ld1 + j;
        u1h[o1] = hh;
        u1l[o1] = ll;
    }
}

// O_b (m x m at O + b*stride_o) -> hi/lo at b*ob + i*ld + j (ld >= m).
// Four consecutive j per thread (8-byte stores) when m and stride_o allow
// 16-byte loads; element by element otherwise.
__global__ __launch_bounds__(256) void split_o_kernel(const float* __restrict__ O, int m, int64_t stride_o,
                                                      uint16_t* __restrict__ oh, uint16_t* __restrict__ ol,
                                                      int64_t ld, int64_t ob, int vec) {
    const int b = blockIdx.z, i = blockIdx.y;
    const float* src = O + (int64_t)b * stride_o + (int64_t)i * m;
    uint16_t* dh = oh + (int64_t)b * ob + (int64_t)i * ld;
    uint16_t* dl = ol + (int64_t)b * ob + (int64_t)i * ld;
    if (vec) {
        for (int j = (blockIdx.x * 256 + threadIdx.x) * 4; j < m; j += gridDim.x * 256 * 4) {
            const f32x4 x = *reinterpret_cast<const f32x4*>(src + j);
            u16x4 hv, lv;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                hv[e] = rne_bf16(x[e]);
                lv[e] = rne_bf16(x[e] - bf16_f32(hv[e]));
            }
            *reinterpret_cast<u16x4*>(dh + j) = hv;
            *reinterpret_cast<u16x4*>(dl + j) = lv;
        }
        return;
    }
    for (int j = blockIdx.x * 256 + threadIdx.x; j < m; j += gridDim.x * 256) {
        const float x = src[j];
        const uint16_t hh = rne_bf16(x);
        dh[j] = hh;
        dl[j] = rne_bf16(x - bf16_f32(hh));
    }
}

inline int64_t pad8(int64_t k) { return (k + 7) / 8 * 8; }
inline size_t al256(size_t n) { return (n + 255) / 256 * 256; }

template <int BI, int KS, bool EPI_T>
hipError_t launch_tile(const Bf16Desc& g, hipStream_t s) {
    const int edge = 64 * BI;
    const int tm = (g.M + edge - 1) / edge, tn = (g.N + edge - 1) / edge;
    const int64_t tiles = (int64_t)tm * tn * g.batch;
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    const char* order = getenv("ROT_BF16_ORDER");
    const int nf = order ? (order[0] == 'n') : 0;
    // with d = 4 the row extent d*mp is a multiple of 4, so every group of
    // four rows is complete and the vector store path covers all of them
    if (EPI_T && g.d == 4)
        hipLaunchKernelGGL((gemm_bf16x3_kernel<BI, BI, KS, EPI_T, true>), dim3((unsigned)tiles), dim3(kThreads), 0, s,
                           g, tm, tn, nf);
    else
        hipLaunchKernelGGL((gemm_bf16x3_kernel<BI, BI, KS, EPI_T, false>), dim3((unsigned)tiles), dim3(kThreads), 0,
                           s, g, tm, tn, nf);
    return hipGetLastError();
}

// 256 x 256 tiles with 32-wide K slices when both output extents reach 256
// (fewer LDS reads per matrix instruction, and a longer multiply phase per
// slice to hide the next slice's HBM latency); else 128 x 128 with 16-wide
// slices.  Environment ROT_BF16_TILE=128 forces the small tile and
// ROT_BF16_KS=16 the narrow slice (measurement knobs).
template <bool EPI_T>
hipError_t launch_bf16(const Bf16Desc& g, hipStream_t s) {
    const char* env = getenv("ROT_BF16_TILE");
    const char* ks = getenv("ROT_BF16_KS");
    const bool small = env && !strcmp(env, "128");
    const bool narrow = ks && !strcmp(ks, "16");
    // the split-transposed epilogue fits the 256 x 256 register budget only in
    // its d = 4 vector-store form
    const bool big_ok = !EPI_T || g.d == 4;
    if (!small && big_ok && g.M >= 256 && g.N >= 256)
        return narrow ? launch_tile<4, 16, EPI_T>(g, s) : launch_tile<4, 32, EPI_T>(g, s);
    return launch_tile<2, 16, EPI_T>(g, s);
}

struct Bf16Layout {
    int64_t ld1, ld2;     // padded K of U1 and O (m) and of U2 / Tt (m*d)
    size_t u1, u2, t_op;  // bytes of one hi (or lo) array
    size_t o_op;          // bytes of one operator's split O (hi or lo)
    size_t shared;        // bytes of the pre-split U (4 arrays)
};

Bf16Layout layout(int m, int d, int mp) {
    Bf16Layout L;
    L.ld1 = pad8(m);
    L.ld2 = pad8((int64_t)m * d);
    L.u1 = al256((size_t)d * mp * L.ld1 * 2);
    L.u2 = al256((size_t)mp * L.ld2 * 2);
    L.t_op = al256((size_t)mp * L.ld2 * 2);
    L.o_op = al256((size_t)m * L.ld1 * 2);
    L.shared = 2 * L.u1 + 2 * L.u2;
    return L;
}

}  // namespace

size_t bf16_group_workspace(int m, int d, int mp, int ops) {
    const Bf16Layout L = layout(m, d, mp);
    return L.shared + (size_t)ops * 2 * (L.t_op + L.o_op);
}

hipError_t rotate_bf16(const rot_problem& p, int b0, int nb, void* ws, hipStream_t stream) {
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
            hipLaunchKernelGGL(split_u_kernel, grid, dim3(256), 0, stream, static_cast<const float*>(p.U), rows,
                               p.mp, p.d, u1h, u1l, L.ld1, u2h, u2l, L.ld2);
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
    }
    // stage 1, transposed: C(beta*d+s, i) = sum_j U1[beta*d+s][j] O_b[i][j] = T_b(i, beta*d+s)
    Bf16Desc a{};
    a.M = p.d * p.mp;
    a.N = p.m;
    a.K = p.m;
    a.batch = nb;
    a.a_hi = u1h;
    a.a_lo = u1l;
    a.lda = L.ld1;
    a.a_bs = 0;
    a.b_hi = oh;
    a.b_lo = ol;
    a.ldb = L.ld1;
    a.b_bs = (int64_t)(L.o_op / 2);
    a.t_hi = th;
    a.t_lo = tl;
    a.d = p.d;
    a.t_ld = L.ld2;
    a.t_bs = (int64_t)(L.t_op / 2);
    hipError_t e = prof_timed("split_o_bf16x3", stream, [&] {
        const float* Ob = static_cast<const float*>(p.O) + (int64_t)b0 * p.stride_o;
        const int vec = (reinterpret_cast<uintptr_t>(Ob) & 15) == 0 && p.m % 4 == 0 && p.stride_o % 4 == 0;
        const dim3 grid((p.m + (vec ? 1023 : 255)) / (vec ? 1024 : 256), p.m, nb);
        hipLaunchKernelGGL(split_o_kernel, grid, dim3(256), 0, stream, Ob, p.m, p.stride_o, oh, ol, L.ld1,
                           (int64_t)(L.o_op / 2), vec);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    e = prof_timed("stage1_bf16x3", stream, [&] { return launch_bf16<true>(a, stream); });
    if (e != hipSuccess) return e;
    // stage 2: out_b[alpha][beta] = sum_r U2[alpha][r] Tt_b[beta][r]
    Bf16Desc b{};
    b.M = p.mp;
    b.N = p.mp;
    b.K = p.m * p.d;
    b.batch = nb;
    b.a_hi = u2h;
    b.a_lo = u2l;
    b.lda = L.ld2;
    b.a_bs = 0;
    b.b_hi = th;
    b.b_lo = tl;
    b.ldb = L.ld2;
    b.b_bs = (int64_t)(L.t_op / 2);
    b.c = static_cast<float*>(p.out) + (int64_t)b0 * p.stride_out;
    b.ldc = p.mp;
    b.c_bs = p.stride_out;
    return prof_timed("stage2_bf16x3", stream, [&] { return launch_bf16<false>(b, stream); });
}

}  // namespace rot
