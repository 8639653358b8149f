// Split-BF16 rotation: every FP32 operand x is carried as x = hi + lo with
// hi = bf16(x), lo = bf16(x - hi) (round to nearest even), and every product
// a*b as a_hi*b_hi + a_hi*b_lo + a_lo*b_hi on BF16 matrix cores with FP32
// accumulation (the dropped a_lo*b_lo term is below 2^-16 relative).
//
// BF16 matrix instructions take 8 consecutive k per lane, so both operands
// are kept K-contiguous:
//   stage 1  T_b = O_b U_r :  A = O_b (FP32, split while staging into LDS),
//            B = U1[beta*d+s][j] = U[j*d+s][beta] (pre-split once per call);
//            the epilogue splits T and stores it transposed,
//            Tt_b[beta][i*d+s] = T_b(i, beta*d+s), i.e. as stage 2's B.
//   stage 2  out_b = U^T T_b :  A = U2[alpha][r] = U[r][alpha] (pre-split),
//            B = Tt_b; FP32 output.
// Stage 1's N index is ordered n = beta*d + s (site state fastest), so that
// one lane's d neighbours hold the d consecutive entries r = i*d + s of Tt.
// Tiles are 256 x 256 (four waves of 128 x 128) so that each 128-bit LDS
// fragment read feeds 3 x 4 matrix instructions.
#include <hip/hip_runtime.h>

#include <algorithm>

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
    // A (M x K, K-contiguous): FP32 (a32) or pre-split (a_hi, a_lo)
    const float* a32;
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
    // split-transposed epilogue: C(i, n = beta*d + s) -> T[beta*t_ld + i*d + s]
    uint16_t* t_hi;
    uint16_t* t_lo;
    int d;
    int64_t t_ld, t_bs;
};

// Stage an R x 16 slice of a pre-split K-contiguous operand into LDS:
// 2 arrays x R rows x 2 chunks of 8 = 4R chunks of 16 bytes.
template <int R>
struct SplitSlice {
    static constexpr int CH = 4 * R / kThreads;
    u16x8 r[CH];
    __device__ inline void load(const uint16_t* __restrict__ hi, const uint16_t* __restrict__ lo, int64_t ld,
                                int r0, int rows, int k0, int ks, int tid) {
#pragma unroll
        for (int c = 0; c < CH; c++) {
            const int f = tid + c * kThreads;  // [0, 4R)
            const int arr = f / (2 * R), q = f % (2 * R);
            const int row = q >> 1, k = (q & 1) * 8;
            const int gr = r0 + row, gk = k0 + k;
            const uint16_t* p = (arr ? lo : hi) + (int64_t)gr * ld + gk;
            if (gr < rows && gk + 8 <= ks) {
                r[c] = *reinterpret_cast<const u16x8*>(p);
            } else {
#pragma unroll
                for (int e = 0; e < 8; e++) r[c][e] = (gr < rows && gk + e < ks) ? p[e] : (uint16_t)0;
            }
        }
    }
    __device__ inline void store(uint16_t* s_hi, uint16_t* s_lo, int tid) const {
#pragma unroll
        for (int c = 0; c < CH; c++) {
            const int f = tid + c * kThreads;
            const int arr = f / (2 * R), q = f % (2 * R);
            const int row = q >> 1, k = (q & 1) * 8;
            *reinterpret_cast<u16x8*>((arr ? s_lo : s_hi) + row * kPitch + k) = r[c];
        }
    }
};

// Stage an R x 16 slice of an FP32 K-contiguous operand, splitting it:
// R rows x 4 chunks of 4 floats.
template <int R, bool VEC>
struct F32Slice {
    static constexpr int CH = 4 * R / kThreads;
    f32x4 r[CH];
    __device__ inline void load(const float* __restrict__ a, int64_t ld, int r0, int rows, int k0, int ks,
                                int tid) {
#pragma unroll
        for (int c = 0; c < CH; c++) {
            const int f = tid + c * kThreads;
            const int row = f >> 2, k = (f & 3) * 4;
            const int gr = r0 + row, gk = k0 + k;
            const float* p = a + (int64_t)gr * ld + gk;
            if (VEC && gr < rows && gk + 4 <= ks) {
                r[c] = *reinterpret_cast<const f32x4*>(p);
            } else {
#pragma unroll
                for (int e = 0; e < 4; e++) r[c][e] = (gr < rows && gk + e < ks) ? p[e] : 0.f;
            }
        }
    }
    __device__ inline void store(uint16_t* s_hi, uint16_t* s_lo, int tid) const {
#pragma unroll
        for (int c = 0; c < CH; c++) {
            const int f = tid + c * kThreads;
            const int row = f >> 2, k = (f & 3) * 4;
            u16x4 h, l;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const uint16_t hh = rne_bf16(r[c][e]);
                h[e] = hh;
                l[e] = rne_bf16(r[c][e] - bf16_f32(hh));
            }
            *reinterpret_cast<u16x4*>(s_hi + row * kPitch + k) = h;
            *reinterpret_cast<u16x4*>(s_lo + row * kPitch + k) = l;
        }
    }
};

template <int R, bool A_F32, bool VEC_A>
struct ASlice;
template <int R, bool VEC_A>
struct ASlice<R, true, VEC_A> : F32Slice<R, VEC_A> {
    __device__ inline void fetch(const Bf16Desc& g, int bidx, int r0, int k0, int tid) {
        this->load(g.a32 + (int64_t)bidx * g.a_bs, g.lda, r0, g.M, k0, g.K, tid);
    }
};
template <int R, bool VEC_A>
struct ASlice<R, false, VEC_A> : SplitSlice<R> {
    __device__ inline void fetch(const Bf16Desc& g, int bidx, int r0, int k0, int tid) {
        this->load(g.a_hi + (int64_t)bidx * g.a_bs, g.a_lo + (int64_t)bidx * g.a_bs, g.lda, r0, g.M, k0, g.K, tid);
    }
};

// Tile BM x BN = (2*BI*32) x (2*BJ*32): four waves in a 2 x 2 grid, each
// BI x BJ blocks of v_mfma_f32_32x32x16_bf16.  That instruction takes from
// lane l A(row l%32, k 8*(l/32)+e) and B(k 8*(l/32)+e, col l%32), e < 8, and
// leaves C(8*(v/4) + 4*(l/32) + v%4, l%32) in accumulator element v.  One
// LDS slice is one k step of 16; its 128-bit fragment reads are
// conflict-free with the 48-byte row pitch.
template <int BI, int BJ, bool A_F32, bool VEC_A, bool EPI_T>
__global__ __launch_bounds__(kThreads, 1) void gemm_bf16x3_kernel(Bf16Desc g, int tiles_m, int tiles_n) {
    constexpr int BM = 64 * BI, BN = 64 * BJ;
    constexpr int A_ARR = BM * kPitch, B_ARR = BN * kPitch;
    constexpr int BUF = 2 * A_ARR + 2 * B_ARR;
    __shared__ __attribute__((aligned(16))) uint16_t lds[2 * BUF];  // per buffer: A_hi, A_lo, B_hi, B_lo

    const int lin = xcd_linear_id();
    const int per_batch = tiles_m * tiles_n;
    const int bidx = lin / per_batch;
    const int rr = lin % per_batch;
    const int m0 = (rr % tiles_m) * BM, n0 = (rr / tiles_m) * BN;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int h = lane >> 5, c = lane & 31;

    ASlice<BM, A_F32, VEC_A> la;
    SplitSlice<BN> lb;
    const uint16_t* bh = g.b_hi + (int64_t)bidx * g.b_bs;
    const uint16_t* bl = g.b_lo + (int64_t)bidx * g.b_bs;
    const int nk = (g.K + kSlice - 1) / kSlice;

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

    la.fetch(g, bidx, m0, 0, tid);
    lb.load(bh, bl, g.ldb, n0, g.N, 0, g.K, tid);
    la.store(A_hi(0), A_lo(0), tid);
    lb.store(B_hi(0), B_lo(0), tid);
    __syncthreads();

    for (int t = 0; t < nk; t++) {
        const int cur = t & 1;
        if (t + 1 < nk) {
            la.fetch(g, bidx, m0, (t + 1) * kSlice, tid);
            lb.load(bh, bl, g.ldb, n0, g.N, (t + 1) * kSlice, g.K, tid);
        }
        bf16x8 ah[BI], al[BI], bhv[BJ], blv[BJ];
#pragma unroll
        for (int i = 0; i < BI; i++) {
            const int ra = (wm * 32 * BI + i * 32 + c) * kPitch + h * 8;
            ah[i] = *reinterpret_cast<const bf16x8*>(A_hi(cur) + ra);
            al[i] = *reinterpret_cast<const bf16x8*>(A_lo(cur) + ra);
        }
#pragma unroll
        for (int j = 0; j < BJ; j++) {
            const int rb = (wn * 32 * BJ + j * 32 + c) * kPitch + h * 8;
            bhv[j] = *reinterpret_cast<const bf16x8*>(B_hi(cur) + rb);
            blv[j] = *reinterpret_cast<const bf16x8*>(B_lo(cur) + rb);
        }
#pragma unroll
        for (int i = 0; i < BI; i++)
#pragma unroll
            for (int k = 0; k < BJ; k++) {
                acc[i][k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bhv[k], acc[i][k], 0, 0, 0);
                acc[i][k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], blv[k], acc[i][k], 0, 0, 0);
                acc[i][k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bhv[k], acc[i][k], 0, 0, 0);
            }
        if (t + 1 < nk) {
            la.store(A_hi(cur ^ 1), A_lo(cur ^ 1), tid);
            lb.store(B_hi(cur ^ 1), B_lo(cur ^ 1), tid);
        }
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < BI; i++)
#pragma unroll
        for (int k = 0; k < BJ; k++) {
            const int col = n0 + wn * 32 * BJ + k * 32 + c;
            if (col >= g.N) continue;
            if (EPI_T) {
                const int beta = col / g.d, s = col % g.d;
                uint16_t* th = g.t_hi + (int64_t)bidx * g.t_bs + (int64_t)beta * g.t_ld + s;
                uint16_t* tl = g.t_lo + (int64_t)bidx * g.t_bs + (int64_t)beta * g.t_ld + s;
#pragma unroll
                for (int v = 0; v < 16; v++) {
                    const int row = m0 + wm * 32 * BI + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
                    if (row < g.M) {
                        const float x = acc[i][k][v];
                        const uint16_t hh = rne_bf16(x);
                        th[(int64_t)row * g.d] = hh;
                        tl[(int64_t)row * g.d] = rne_bf16(x - bf16_f32(hh));
                    }
                }
            } else {
                float* cb = g.c + (int64_t)bidx * g.c_bs;
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

inline int64_t pad8(int64_t k) { return (k + 7) / 8 * 8; }
inline size_t al256(size_t n) { return (n + 255) / 256 * 256; }

template <int BI, bool A_F32, bool VEC_A, bool EPI_T>
hipError_t launch_tile(const Bf16Desc& g, hipStream_t s) {
    const int edge = 64 * BI;
    const int tm = (g.M + edge - 1) / edge, tn = (g.N + edge - 1) / edge;
    const int64_t tiles = (int64_t)tm * tn * g.batch;
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gemm_bf16x3_kernel<BI, BI, A_F32, VEC_A, EPI_T>), dim3((unsigned)tiles), dim3(kThreads),
                       0, s, g, tm, tn);
    return hipGetLastError();
}

// 256 x 256 tiles when both output extents reach 256, else 128 x 128.
template <bool A_F32, bool VEC_A, bool EPI_T>
hipError_t launch_bf16(const Bf16Desc& g, hipStream_t s) {
    if (g.M >= 256 && g.N >= 256) return launch_tile<4, A_F32, VEC_A, EPI_T>(g, s);
    return launch_tile<2, A_F32, VEC_A, EPI_T>(g, s);
}

struct Bf16Layout {
    int64_t ld1, ld2;     // padded K of U1 (m) and of U2 / Tt (m*d)
    size_t u1, u2, t_op;  // bytes of one hi (or lo) array
    size_t shared;        // bytes of the pre-split U (4 arrays)
};

Bf16Layout layout(int m, int d, int mp) {
    Bf16Layout L;
    L.ld1 = pad8(m);
    L.ld2 = pad8((int64_t)m * d);
    L.u1 = al256((size_t)d * mp * L.ld1 * 2);
    L.u2 = al256((size_t)mp * L.ld2 * 2);
    L.t_op = al256((size_t)mp * L.ld2 * 2);
    L.shared = 2 * L.u1 + 2 * L.u2;
    return L;
}

}  // namespace

size_t bf16_group_workspace(int m, int d, int mp, int ops) {
    const Bf16Layout L = layout(m, d, mp);
    return L.shared + (size_t)ops * 2 * L.t_op;
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
    // stage 1: T_b(i, beta*d+s) = sum_j O_b[i][j] U[j*d+s][beta]
    Bf16Desc a{};
    a.M = p.m;
    a.N = p.d * p.mp;
    a.K = p.m;
    a.batch = nb;
    a.a32 = static_cast<const float*>(p.O) + (int64_t)b0 * p.stride_o;
    a.lda = p.m;
    a.a_bs = p.stride_o;
    a.b_hi = u1h;
    a.b_lo = u1l;
    a.ldb = L.ld1;
    a.b_bs = 0;
    a.t_hi = th;
    a.t_lo = tl;
    a.d = p.d;
    a.t_ld = L.ld2;
    a.t_bs = (int64_t)(L.t_op / 2);
    const bool vec = (reinterpret_cast<uintptr_t>(a.a32) & 15) == 0 && p.m % 4 == 0 && p.stride_o % 4 == 0;
    hipError_t e = prof_timed("stage1_bf16x3", stream, [&] {
        return vec ? launch_bf16<true, true, true>(a, stream) : launch_bf16<true, false, true>(a, stream);
    });
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
    return prof_timed("stage2_bf16x3", stream, [&] { return launch_bf16<false, true, false>(b, stream); });
}

}  // namespace rot
