// The system's reduced density matrix per quantum-number sector, its
// eigenbasis, and the choice of the kept states (Sec. 2: Eq. (2), step 4,
// Eq. (3)), all in FP64.
//
// rho_k = psi_k psi_k^T is formed tile by tile into a zero-padded n_pad x n_pad
// matrix (n_pad a multiple of 64) and diagonalised by two-sided block Jacobi:
// the matrix is cut into 32-wide blocks; in each round the blocks are paired
// by the circle method, every pair's 64 x 64 principal submatrix is swept once
// by scalar Jacobi in LDS (one workgroup per pair, the 32 disjoint rotations
// of a step applied together), and the accumulated 64 x 64 rotations Q are
// applied to the rest of the matrix (A_{P1,P2} <- Q1^T A_{P1,P2} Q2 for every
// two pairs) and to the eigenvector matrix (V_{:,P} <- V_{:,P} Q).  Padded
// rows and columns are exactly zero and never rotate, so they stay decoupled.
// A sector is finished after a full cycle of rounds without any rotation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "rot_internal.h"

namespace rot {

namespace {

constexpr int kBlk = 32;        // Jacobi block edge
constexpr int kPair = 64;       // two blocks
constexpr int kLs = kPair + 1;  // LDS row stride (doubles)
constexpr int kMaxSweeps = 80;
constexpr int kSortMax = 4096;  // largest sector (states)

struct DmSector {
    int n, r, npad, nb;
    const double* psi;
    int64_t ld_psi;
    double* w;
    double* V;
    int64_t ld_v;
    int64_t a_off;  // doubles, into the working matrix and the eigenvector matrix
    int64_t q_off;  // doubles, into the pair rotations (nb/2 blocks of 64 x 64)
    int64_t w_off;  // doubles, into the concatenated sorted eigenvalues
    int flag_off;   // ints, into the per-pair rotation flags
    int pad;
};

struct DmState {
    double floor;  // |a_pq| <= floor counts as zero
    int quiet;     // consecutive rounds without a rotation
    int converged;
    int rounds;
    int pad;
};

struct DmItem {
    int sec, a, b, kind;
};

enum : int { kItemA = 0, kItemV = 1, kItemBook = 2 };

// Round t of the circle method for nb players (nb even): player 0 is fixed,
// players 1..nb-1 sit on a circle turned by t; pair k is (0, c_0) for k = 0
// and (c_k, c_{nb-1-k}) otherwise, with c_j = 1 + (j + t) mod (nb - 1).  Over
// nb - 1 consecutive rounds every two players meet once.  Returns i < j.
__host__ __device__ inline void circle_pair(int nb, int t, int k, int& i, int& j) {
    const int m = nb - 1;
    t %= m;
    int a, b;
    if (k == 0) {
        a = 0;
        b = 1 + t;
    } else {
        a = 1 + (k + t) % m;
        b = 1 + (m - k + t) % m;
    }
    i = a < b ? a : b;
    j = a < b ? b : a;
}

// Global row of local index l (0..63) of the pair of blocks (I, J).
__device__ inline int pair_row(int I, int J, int l) { return l < kBlk ? I * kBlk + l : J * kBlk + (l - kBlk); }

// ---------------------------------------------------------------------------
// rho tile (ti, tj), ti <= tj, of sector it.sec: rho[x][y] = sum_k psi[x][k] psi[y][k]
// over 64 x 64 outputs (4 x 4 per thread), K in slices of 16 through LDS;
// written to both (ti, tj) and its mirror.  The eigenvector matrix is set to
// the identity on the same tiles.
__global__ __launch_bounds__(256) void dm_rho_kernel(const DmSector* __restrict__ secs,
                                                     const DmItem* __restrict__ items, double* __restrict__ A,
                                                     double* __restrict__ Vw) {
    const DmItem it = items[blockIdx.x];
    const DmSector s = secs[it.sec];
    const int ti = it.a, tj = it.b;
    __shared__ double pa[16][kPair + 1];
    __shared__ double pb[16][kPair + 1];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    double acc[4][4];
#pragma unroll
    for (int p = 0; p < 4; p++)
#pragma unroll
        for (int q = 0; q < 4; q++) acc[p][q] = 0.0;
    for (int k0 = 0; k0 < s.r; k0 += 16) {
        for (int e = tid; e < kPair * 16; e += 256) {
            const int row = e >> 4, kk = e & 15;
            const int gi = ti * kPair + row, gj = tj * kPair + row, gk = k0 + kk;
            const bool kin = gk < s.r;
            pa[kk][row] = (kin && gi < s.n) ? s.psi[(int64_t)gi * s.ld_psi + gk] : 0.0;
            pb[kk][row] = (kin && gj < s.n) ? s.psi[(int64_t)gj * s.ld_psi + gk] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 16; kk++) {
            double a[4], b[4];
#pragma unroll
            for (int p = 0; p < 4; p++) a[p] = pa[kk][ty * 4 + p];
#pragma unroll
            for (int q = 0; q < 4; q++) b[q] = pb[kk][tx * 4 + q];
#pragma unroll
            for (int p = 0; p < 4; p++)
#pragma unroll
                for (int q = 0; q < 4; q++) acc[p][q] = fma(a[p], b[q], acc[p][q]);
        }
        __syncthreads();
    }
    double* a = A + s.a_off;
    double* v = Vw + s.a_off;
    const int64_t np = s.npad;
#pragma unroll
    for (int p = 0; p < 4; p++) {
        const int64_t row = ti * kPair + ty * 4 + p;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int64_t col = tj * kPair + tx * 4 + q;
            a[row * np + col] = acc[p][q];
            v[row * np + col] = row == col ? 1.0 : 0.0;
            if (ti != tj) {
                a[col * np + row] = acc[p][q];
                v[col * np + row] = 0.0;
            }
        }
    }
}

// Per sector: the threshold 2^-52 tr(rho) (trace summed in a fixed order) and
// cleared convergence counters.
__global__ __launch_bounds__(256) void dm_prep_kernel(const DmSector* __restrict__ secs,
                                                      const double* __restrict__ A, DmState* __restrict__ st) {
    const DmSector s = secs[blockIdx.x];
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < s.n; i += 256) acc += A[s.a_off + (int64_t)i * s.npad + i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        DmState x;
        x.floor = ldexp(red[0], -52);
        x.quiet = 0;
        x.converged = 0;
        x.rounds = 0;
        x.pad = 0;
        st[blockIdx.x] = x;
    }
}

// ---------------------------------------------------------------------------
// One Jacobi sweep over the 64 x 64 principal submatrix of pair k of round t:
// 63 steps of 32 disjoint rotations (circle order over the 64 local indices).
// Rotation (p, q) with tau = (a_qq - a_pp) / (2 a_pq), t = sign(tau) /
// (|tau| + sqrt(1 + tau^2)), c = 1/sqrt(1 + t^2), s = t c zeroes a_pq of
// J^T A J, J = [[c, s], [-s, c]] on rows/columns (p, q).  Each 2 x 2 block
// (kx <= ky) of the step's pairs is rotated once, so the submatrix stays exactly
// symmetric.  Schedule per step: all 528 blocks are rotated (one per thread),
// then wave 0 derives the next step's rotations while the other waves apply
// this step's to the accumulated Q (parameters double-buffered).
constexpr int kPairThreads = 1024;
constexpr int kSteps = kPair - 1;
constexpr int kBlocks2 = 32 * 33 / 2;

struct Rot2 {
    double c, s, t;
};

__device__ inline Rot2 jacobi_rotation(double app, double aqq, double apq, double floor) {
    Rot2 r{1.0, 0.0, 0.0};
    if (fabs(apq) > floor) {
        const double tau = (aqq - app) / (2.0 * apq);
        r.t = fabs(tau) > 1e150 ? 0.5 / tau : copysign(1.0, tau) / (fabs(tau) + sqrt(1.0 + tau * tau));
        r.c = 1.0 / sqrt(1.0 + r.t * r.t);
        r.s = r.t * r.c;
    }
    return r;
}

// S is held as its upper triangle (entry (a, b) and (b, a) at su(min, max)):
// at every step each unordered pair of indices lies in exactly one 2 x 2
// block, so no mirrored copy has to be written.  Q is held transposed, row
// stride kLq, so a rotation of columns (p, q) of Q updates two rows of Q^T
// with 16-byte LDS accesses.
constexpr int kLq = kPair + 2;

__device__ inline int su(int a, int b) { return a < b ? a * kLs + b : b * kLs + a; }

__global__ __launch_bounds__(kPairThreads) void dm_pair_kernel(const DmSector* __restrict__ secs,
                                                               const DmItem* __restrict__ items,
                                                               double* __restrict__ A, double* __restrict__ Qw,
                                                               const DmState* __restrict__ st,
                                                               int* __restrict__ rotated, int round) {
    const DmItem it = items[blockIdx.x];
    const DmSector s = secs[it.sec];
    const int k = it.a;
    const int tid = threadIdx.x;
    int* flag = rotated + s.flag_off + k;
    if (st[it.sec].converged) {
        if (tid == 0) *flag = 0;
        return;
    }
    const double floor = st[it.sec].floor;
    int I, J;
    circle_pair(s.nb, round, k, I, J);
    __shared__ double S[kPair * kLs];
    __shared__ __attribute__((aligned(16))) double Qt[kPair * kLq];
    __shared__ double rc[2][32], rs[2][32], rt[2][32];
    __shared__ unsigned char tp[kSteps][32], tq[kSteps][32];
    __shared__ int any;
    double* a = A + s.a_off;
    const int64_t np = s.npad;
    {
        constexpr int kPer = kPair * kPair / kPairThreads;
        double sv[kPer];
#pragma unroll
        for (int j = 0; j < kPer; j++) {
            const int e = tid + kPairThreads * j, x = e >> 6, y = e & 63;
            sv[j] = a[(int64_t)pair_row(I, J, x) * np + pair_row(I, J, y)];
        }
#pragma unroll
        for (int j = 0; j < kPer; j++) {
            const int e = tid + kPairThreads * j, x = e >> 6, y = e & 63;
            if (x <= y) S[x * kLs + y] = sv[j];
            Qt[x * kLq + y] = x == y ? 1.0 : 0.0;
        }
    }
    for (int e = tid; e < kSteps * 32; e += kPairThreads) {
        int p, q;
        circle_pair(kPair, e >> 5, e & 31, p, q);
        tp[e >> 5][e & 31] = (unsigned char)p;
        tq[e >> 5][e & 31] = (unsigned char)q;
    }
    if (tid == 0) any = 0;
    __syncthreads();
    if (tid < 32) {
        const int p = tp[0][tid], q = tq[0][tid];
        const Rot2 r = jacobi_rotation(S[p * kLs + p], S[q * kLs + q], S[p * kLs + q], floor);
        rc[0][tid] = r.c;
        rs[0][tid] = r.s;
        rt[0][tid] = r.t;
        if (r.s != 0.0) any = 1;
    }
    // this thread's 2 x 2 block: b = ky (ky + 1) / 2 + kx, kx <= ky
    int kx = 0, ky = 0;
    if (tid < kBlocks2) {
        ky = (int)((sqrtf(8.0f * tid + 1.0f) - 1.0f) * 0.5f);
        while (ky * (ky + 1) / 2 > tid) ky--;
        while ((ky + 1) * (ky + 2) / 2 <= tid) ky++;
        kx = tid - ky * (ky + 1) / 2;
    }
    __syncthreads();
    for (int u = 0; u < kSteps; u++) {
        const int cur = u & 1;
        if (tid < kBlocks2) {
            const int px = tp[u][kx], qx = tq[u][kx];  // px < qx
            if (kx == ky) {
                const double t = rt[cur][kx];
                if (t != 0.0) {
                    const double apq = S[px * kLs + qx];
                    S[px * kLs + px] -= t * apq;
                    S[qx * kLs + qx] += t * apq;
                    S[px * kLs + qx] = 0.0;
                }
            } else {
                const double sx = rs[cur][kx], sy = rs[cur][ky];
                if (sx != 0.0 || sy != 0.0) {
                    const int py = tp[u][ky], qy = tq[u][ky];
                    const double cx = rc[cur][kx], cy = rc[cur][ky];
                    const int iu = su(px, py), iv = su(px, qy), ix = su(qx, py), iy = su(qx, qy);
                    const double u0 = S[iu], v0 = S[iv], x0 = S[ix], y0 = S[iy];
                    const double u1 = cx * u0 - sx * x0, x1 = sx * u0 + cx * x0;
                    const double v1 = cx * v0 - sx * y0, y1 = sx * v0 + cx * y0;
                    S[iu] = cy * u1 - sy * v1;
                    S[iv] = sy * u1 + cy * v1;
                    S[ix] = cy * x1 - sy * y1;
                    S[iy] = sy * x1 + cy * y1;
                }
            }
        }
        __syncthreads();
        if (tid < 64) {
            if (tid < 32 && u + 1 < kSteps) {
                const int p = tp[u + 1][tid], q = tq[u + 1][tid];
                const Rot2 r = jacobi_rotation(S[p * kLs + p], S[q * kLs + q], S[p * kLs + q], floor);
                rc[cur ^ 1][tid] = r.c;
                rs[cur ^ 1][tid] = r.s;
                rt[cur ^ 1][tid] = r.t;
                if (r.s != 0.0) any = 1;
            }
        } else {
            // Q <- Q J: rows p, q of Q^T, two entries per access; 32 pairs x 32
            // row pairs over the 960 threads past wave 0
            for (int wq = tid - 64; wq < 32 * 32; wq += kPairThreads - 64) {
                const int kq = wq >> 5, rq2 = wq & 31;
                const double sn = rs[cur][kq];
                if (sn == 0.0) continue;
                const double c = rc[cur][kq];
                double2* rp = reinterpret_cast<double2*>(Qt + tp[u][kq] * kLq) + rq2;
                double2* rq = reinterpret_cast<double2*>(Qt + tq[u][kq] * kLq) + rq2;
                const double2 vp = *rp, vq = *rq;
                *rp = double2{c * vp.x - sn * vq.x, c * vp.y - sn * vq.y};
                *rq = double2{sn * vp.x + c * vq.x, sn * vp.y + c * vq.y};
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < kPair * kPair; e += kPairThreads) {
        const int x = e >> 6, y = e & 63;
        a[(int64_t)pair_row(I, J, x) * np + pair_row(I, J, y)] = S[su(x, y)];
        Qw[s.q_off + (int64_t)k * kPair * kPair + e] = Qt[y * kLq + x];
    }
    if (tid == 0) *flag = any;
}

typedef double dm_f64x4 __attribute__((ext_vector_type(4)));

// Y = op(L) * R (64 x 64, op(L) = L or L^T, operands in LDS with row stride
// kLs) on v_mfma_f64_16x16x4f64: wave w owns rows 32 (w / 2) .. and columns
// 32 (w % 2) .. as 2 x 2 blocks of 16 x 16.  Lane l supplies A(row l%16, k l/16)
// and B(k l/16, col l%16); element v of block (bi, bj) is row
// 32 wr + 16 bi + 4 v + l/16, column 32 wc + 16 bj + l%16.
template <bool kTransL>
__device__ inline void mm64(const double* L, const double* R, dm_f64x4 (&acc)[2][2], int wr, int wc, int h,
                            int c) {
#pragma unroll
    for (int bi = 0; bi < 2; bi++)
#pragma unroll
        for (int bj = 0; bj < 2; bj++) acc[bi][bj] = dm_f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k4 = 0; k4 < kPair / 4; k4++) {
        const int k = 4 * k4 + h;
        double a[2], b[2];
#pragma unroll
        for (int bi = 0; bi < 2; bi++) {
            const int row = 32 * wr + 16 * bi + c;
            a[bi] = kTransL ? L[k * kLs + row] : L[row * kLs + k];
        }
#pragma unroll
        for (int bj = 0; bj < 2; bj++) b[bj] = R[k * kLs + 32 * wc + 16 * bj + c];
#pragma unroll
        for (int bi = 0; bi < 2; bi++)
#pragma unroll
            for (int bj = 0; bj < 2; bj++)
                acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
    }
}

__device__ inline void acc_to_lds(double* X, const dm_f64x4 (&acc)[2][2], int wr, int wc, int h, int c) {
#pragma unroll
    for (int bi = 0; bi < 2; bi++)
#pragma unroll
        for (int bj = 0; bj < 2; bj++) {
            const int col = 32 * wc + 16 * bj + c;
            X[(32 * wr + 16 * bi + h) * kLs + col] = acc[bi][bj].x;
            X[(32 * wr + 16 * bi + 4 + h) * kLs + col] = acc[bi][bj].y;
            X[(32 * wr + 16 * bi + 8 + h) * kLs + col] = acc[bi][bj].z;
            X[(32 * wr + 16 * bi + 12 + h) * kLs + col] = acc[bi][bj].w;
        }
}

// Applies the rotations of round t: A_{P1,P2} <- Q1^T A_{P1,P2} Q2 for pairs
// P1 < P2 (written with its mirror), V_{R,P} <- V_{R,P} Q_P for every 64-row
// tile R, and per sector the bookkeeping of quiet rounds.
__global__ __launch_bounds__(256) void dm_update_kernel(const DmSector* __restrict__ secs,
                                                        const DmItem* __restrict__ items, double* __restrict__ A,
                                                        double* __restrict__ Vw, const double* __restrict__ Qw,
                                                        DmState* __restrict__ st, const int* __restrict__ rotated,
                                                        int round) {
    const DmItem it = items[blockIdx.x];
    const DmSector s = secs[it.sec];
    const int* rf = rotated + s.flag_off;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1, h = lane >> 4, c = lane & 15;
    if (it.kind == kItemBook) {
        if (tid == 0) {
            DmState x = st[it.sec];
            if (!x.converged) {
                int any = 0;
                for (int k = 0; k < s.nb / 2; k++) any |= rf[k];
                x.rounds++;
                if (any) {
                    x.quiet = 0;
                } else if (++x.quiet >= s.nb - 1) {
                    x.converged = 1;
                }
                st[it.sec] = x;
            }
        }
        return;
    }
    __shared__ double X[kPair * kLs];
    __shared__ double L[kPair * kLs];
    __shared__ double R[kPair * kLs];
    const int64_t np = s.npad;
    dm_f64x4 y[2][2];
    if (it.kind == kItemA) {
        const int P1 = it.a, P2 = it.b;
        const int r1 = rf[P1], r2 = rf[P2];
        if (!r1 && !r2) return;
        int I1, J1, I2, J2;
        circle_pair(s.nb, round, P1, I1, J1);
        circle_pair(s.nb, round, P2, I2, J2);
        double* a = A + s.a_off;
        const double* q1 = Qw + s.q_off + (int64_t)P1 * kPair * kPair;
        const double* q2 = Qw + s.q_off + (int64_t)P2 * kPair * kPair;
        // all loads of a thread issued before the first LDS write
        double xv[16], lv[16], rv[16];
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const int e = tid + 256 * j, x = e >> 6, z = e & 63;
            xv[j] = a[(int64_t)pair_row(I1, J1, x) * np + pair_row(I2, J2, z)];
            lv[j] = r1 ? q1[e] : 0.0;
            rv[j] = r2 ? q2[e] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const int e = tid + 256 * j, x = e >> 6, z = e & 63;
            X[x * kLs + z] = xv[j];
            L[x * kLs + z] = lv[j];
            R[x * kLs + z] = rv[j];
        }
        __syncthreads();
        if (r2) {
            mm64<false>(X, R, y, wr, wc, h, c);
            __syncthreads();
            acc_to_lds(X, y, wr, wc, h, c);
            __syncthreads();
        }
        if (r1) {
            mm64<true>(L, X, y, wr, wc, h, c);
            __syncthreads();
            acc_to_lds(X, y, wr, wc, h, c);
            __syncthreads();
        }
        // the block and its mirror, both written along rows
        for (int e = tid; e < kPair * kPair; e += 256) {
            const int x = e >> 6, z = e & 63;
            a[(int64_t)pair_row(I1, J1, x) * np + pair_row(I2, J2, z)] = X[x * kLs + z];
            a[(int64_t)pair_row(I2, J2, x) * np + pair_row(I1, J1, z)] = X[z * kLs + x];
        }
        return;
    }
    // kItemV: rows it.a * 64 .. +64 of V, columns of pair it.b
    const int P = it.b;
    if (!rf[P]) return;
    int I, J;
    circle_pair(s.nb, round, P, I, J);
    double* v = Vw + s.a_off;
    const double* qm = Qw + s.q_off + (int64_t)P * kPair * kPair;
    const int64_t r0 = (int64_t)it.a * kPair;
    double xv[16], rv[16];
#pragma unroll
    for (int j = 0; j < 16; j++) {
        const int e = tid + 256 * j, x = e >> 6, z = e & 63;
        xv[j] = v[(r0 + x) * np + pair_row(I, J, z)];
        rv[j] = qm[e];
    }
#pragma unroll
    for (int j = 0; j < 16; j++) {
        const int e = tid + 256 * j, x = e >> 6, z = e & 63;
        X[x * kLs + z] = xv[j];
        R[x * kLs + z] = rv[j];
    }
    __syncthreads();
    mm64<false>(X, R, y, wr, wc, h, c);
#pragma unroll
    for (int bi = 0; bi < 2; bi++)
#pragma unroll
        for (int bj = 0; bj < 2; bj++) {
            const int64_t col = pair_row(I, J, 32 * wc + 16 * bj + c);
            const int64_t row = r0 + 32 * wr + 16 * bi + h;
            v[row * np + col] = y[bi][bj].x;
            v[(row + 4) * np + col] = y[bi][bj].y;
            v[(row + 8) * np + col] = y[bi][bj].z;
            v[(row + 12) * np + col] = y[bi][bj].w;
        }
}

__global__ __launch_bounds__(256) void dm_count_kernel(const DmState* __restrict__ st, int n_sec,
                                                       int* __restrict__ out) {
    __shared__ int red[256];
    int c = 0;
    for (int k = threadIdx.x; k < n_sec; k += 256) c += st[k].converged ? 0 : 1;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// ---------------------------------------------------------------------------
// Per sector: the diagonal sorted descending (equal values by position, a
// bitonic network in LDS), written to w and to the concatenated list, and the
// eigenvector columns gathered in that order into the caller's V.
__device__ inline bool dm_before(double ka, int ia, double kb, int ib) {
    return ka > kb || (ka == kb && ia < ib);
}

__global__ __launch_bounds__(256) void dm_sort_kernel(const DmSector* __restrict__ secs,
                                                      const double* __restrict__ A, const double* __restrict__ Vw,
                                                      double* __restrict__ wall) {
    const DmSector s = secs[blockIdx.x];
    __shared__ double key[kSortMax];
    __shared__ int idx[kSortMax];
    const int tid = threadIdx.x;
    int p2 = 1;
    while (p2 < s.n) p2 <<= 1;
    for (int i = tid; i < p2; i += 256) {
        key[i] = i < s.n ? A[s.a_off + (int64_t)i * s.npad + i] + 0.0 : -INFINITY;
        idx[i] = i;
    }
    __syncthreads();
    for (int size = 2; size <= p2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < p2; i += 256) {
                const int j = i ^ stride;
                if (j <= i) continue;
                const bool up = (i & size) == 0;
                const bool sw = up ? dm_before(key[j], idx[j], key[i], idx[i])
                                   : dm_before(key[i], idx[i], key[j], idx[j]);
                if (sw) {
                    const double tk = key[i];
                    key[i] = key[j];
                    key[j] = tk;
                    const int tj = idx[i];
                    idx[i] = idx[j];
                    idx[j] = tj;
                }
            }
            __syncthreads();
        }
    }
    for (int k = tid; k < s.n; k += 256) {
        s.w[k] = key[k];
        wall[s.w_off + k] = key[k];
    }
    const double* v = Vw + s.a_off;
    for (int64_t e = tid; e < (int64_t)s.n * s.n; e += 256) {
        const int64_t row = e / s.n;
        const int col = (int)(e - row * s.n);
        // idx[col] < n for finite diagonals; the clamp keeps the read in the
        // sector's block should a non-finite value reorder the padding
        const int src = idx[col] < s.n ? idx[col] : col;
        s.V[row * s.ld_v + col] = v[row * s.npad + src];
    }
}

// Eigenvalues as unsigned keys with the same order (negative zero counts as zero).
__device__ inline uint64_t dm_key(double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x + 0.0);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// Number of leading entries of a descending list whose key is >= c.
__device__ inline int dm_count_ge(const double* w, int n, uint64_t c) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (dm_key(w[mid]) >= c) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// The m_keep largest eigenvalues over all sectors: the m_keep-th largest key T
// found bit by bit (largest T with #(key >= T) >= m_keep; each thread counts
// its share of the concatenated lists, held in registers when they fit), all
// entries above T kept, entries equal to T handed out in sector order; then
// the weight left out, per sector by one wave (strided lanes, then a fixed
// butterfly) and over sectors in sector order.
constexpr int kSelThreads = 1024;
constexpr int kSelWaves = kSelThreads / 64;
constexpr int kSelCache = 16;

__global__ __launch_bounds__(kSelThreads) void dm_select_kernel(const DmSector* __restrict__ secs, int n_sec,
                                                                const double* __restrict__ wall, int64_t m_keep,
                                                                int64_t total, int* __restrict__ above,
                                                                int* __restrict__ equal, double* __restrict__ part,
                                                                int32_t* __restrict__ kept,
                                                                double* __restrict__ eps) {
    __shared__ long long red[2][kSelWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (m_keep >= total || m_keep == 0) {
        for (int k = tid; k < n_sec; k += kSelThreads) kept[k] = m_keep == 0 ? 0 : secs[k].n;
    } else {
        const bool cached = total <= (int64_t)kSelThreads * kSelCache;
        uint64_t kc[kSelCache];
#pragma unroll
        for (int j = 0; j < kSelCache; j++) {
            const int64_t e = tid + (int64_t)kSelThreads * j;
            kc[j] = (cached && e < total) ? dm_key(wall[e]) : 0;  // key 0 is never counted (c >= 1)
        }
        uint64_t T = 0;
        for (int bit = 63; bit >= 0; bit--) {
            const uint64_t c = T | (1ull << bit);
            int cnt = 0;
            if (cached) {
#pragma unroll
                for (int j = 0; j < kSelCache; j++) cnt += kc[j] >= c ? 1 : 0;
            } else {
                for (int64_t e = tid; e < total; e += kSelThreads) cnt += dm_key(wall[e]) >= c ? 1 : 0;
            }
            for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
            const int buf = bit & 1;
            if (lane == 0) red[buf][wave] = cnt;
            __syncthreads();
            long long tot = 0;
            for (int w = 0; w < kSelWaves; w++) tot += red[buf][w];
            if (tot >= m_keep) T = c;
        }
        for (int k = tid; k < n_sec; k += kSelThreads) {
            const double* w = wall + secs[k].w_off;
            const int ge = dm_count_ge(w, secs[k].n, T);
            const int gt = T == ~0ull ? 0 : dm_count_ge(w, secs[k].n, T + 1);
            above[k] = gt;
            equal[k] = ge - gt;
        }
        __syncthreads();
        if (tid == 0) {
            long long need = m_keep;
            for (int k = 0; k < n_sec; k++) need -= above[k];
            for (int k = 0; k < n_sec; k++) {
                const long long take = need < equal[k] ? need : equal[k];
                kept[k] = above[k] + (int)take;
                need -= take;
            }
        }
    }
    __syncthreads();
    for (int k = wave; k < n_sec; k += kSelWaves) {
        const double* w = wall + secs[k].w_off;
        double acc = 0.0;
        for (int i = kept[k] + lane; i < secs[k].n; i += 64) acc += w[i];
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane == 0) part[k] = acc;
    }
    __syncthreads();
    if (tid == 0) {
        double acc = 0.0;
        for (int k = 0; k < n_sec; k++) acc += part[k];
        eps[0] = acc;
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct DmLayout {
    std::vector<DmSector> secs;
    std::vector<DmItem> rho_items, pair_items, upd_items;
    size_t off_secs, off_state, off_rho, off_pair, off_upd, off_flags, off_count, off_above, off_equal, off_part;
    size_t off_A, off_V, off_Q, off_W, total;
    int max_rounds;  // rounds per sweep: max over sectors of nb - 1
};

DmLayout dm_layout(const rot_dm_sector* in, int n_sec) {
    DmLayout L;
    int64_t a_off = 0, q_off = 0, w_off = 0;
    int flag_off = 0;
    L.max_rounds = 1;
    for (int k = 0; k < n_sec; k++) {
        DmSector s{};
        s.n = in[k].n;
        s.r = in[k].r;
        s.npad = (s.n + kPair - 1) / kPair * kPair;
        s.nb = s.npad / kBlk;
        s.psi = in[k].psi;
        s.ld_psi = in[k].ld_psi;
        s.w = in[k].w;
        s.V = in[k].V;
        s.ld_v = in[k].ld_v;
        s.a_off = a_off;
        s.q_off = q_off;
        s.w_off = w_off;
        s.flag_off = flag_off;
        const int h = s.nb / 2, tiles = s.npad / kPair;
        a_off += (int64_t)s.npad * s.npad;
        q_off += (int64_t)h * kPair * kPair;
        w_off += s.n;
        flag_off += h;
        L.max_rounds = std::max(L.max_rounds, s.nb - 1);
        for (int j = 0; j < tiles; j++)
            for (int i = 0; i <= j; i++) L.rho_items.push_back({k, i, j, 0});
        for (int p = 0; p < h; p++) L.pair_items.push_back({k, p, 0, 0});
        for (int p2 = 0; p2 < h; p2++)
            for (int p1 = 0; p1 < p2; p1++) L.upd_items.push_back({k, p1, p2, kItemA});
        for (int rt = 0; rt < tiles; rt++)
            for (int p = 0; p < h; p++) L.upd_items.push_back({k, rt, p, kItemV});
        L.upd_items.push_back({k, 0, 0, kItemBook});
        L.secs.push_back(s);
    }
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    L.off_secs = take(sizeof(DmSector) * n_sec);
    L.off_rho = take(sizeof(DmItem) * L.rho_items.size());
    L.off_pair = take(sizeof(DmItem) * L.pair_items.size());
    L.off_upd = take(sizeof(DmItem) * L.upd_items.size());
    L.off_state = take(sizeof(DmState) * n_sec);
    L.off_flags = take(sizeof(int) * (size_t)std::max(flag_off, 1));
    L.off_count = take(sizeof(int));
    L.off_above = take(sizeof(int) * n_sec);
    L.off_equal = take(sizeof(int) * n_sec);
    L.off_part = take(sizeof(double) * n_sec);
    L.off_A = take(sizeof(double) * (size_t)a_off);
    L.off_V = take(sizeof(double) * (size_t)a_off);
    L.off_Q = take(sizeof(double) * (size_t)q_off);
    L.off_W = take(sizeof(double) * (size_t)std::max<int64_t>(w_off, 1));
    L.total = o;
    return L;
}

}  // namespace

size_t density_workspace_bytes(const rot_dm_sector* sectors, int n_sectors) {
    return dm_layout(sectors, n_sectors).total;
}

hipError_t density_basis(const rot_dm_sector* sectors, int n_sec, int64_t m_keep, int32_t* kept, double* eps,
                         void* workspace, hipStream_t stream, bool* converged) {
    DmLayout L = dm_layout(sectors, n_sec);
    char* ws = static_cast<char*>(workspace);
    // host tables -> workspace head (one copy; the host buffer outlives it: the
    // first convergence check below synchronises the stream)
    std::vector<char> head(L.off_state, 0);
    std::memcpy(head.data() + L.off_secs, L.secs.data(), sizeof(DmSector) * n_sec);
    std::memcpy(head.data() + L.off_rho, L.rho_items.data(), sizeof(DmItem) * L.rho_items.size());
    std::memcpy(head.data() + L.off_pair, L.pair_items.data(), sizeof(DmItem) * L.pair_items.size());
    std::memcpy(head.data() + L.off_upd, L.upd_items.data(), sizeof(DmItem) * L.upd_items.size());
    hipError_t e = hipMemcpyAsync(ws, head.data(), head.size(), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return e;
    const DmSector* secs = reinterpret_cast<const DmSector*>(ws + L.off_secs);
    const DmItem* rho_items = reinterpret_cast<const DmItem*>(ws + L.off_rho);
    const DmItem* pair_items = reinterpret_cast<const DmItem*>(ws + L.off_pair);
    const DmItem* upd_items = reinterpret_cast<const DmItem*>(ws + L.off_upd);
    DmState* st = reinterpret_cast<DmState*>(ws + L.off_state);
    int* flags = reinterpret_cast<int*>(ws + L.off_flags);
    int* count = reinterpret_cast<int*>(ws + L.off_count);
    double* A = reinterpret_cast<double*>(ws + L.off_A);
    double* Vw = reinterpret_cast<double*>(ws + L.off_V);
    double* Qw = reinterpret_cast<double*>(ws + L.off_Q);
    double* W = reinterpret_cast<double*>(ws + L.off_W);

    e = prof_timed("dm_rho", stream, [&] {
        hipLaunchKernelGGL(dm_rho_kernel, dim3((unsigned)L.rho_items.size()), dim3(256), 0, stream, secs,
                           rho_items, A, Vw);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(dm_prep_kernel, dim3(n_sec), dim3(256), 0, stream, secs, (const double*)A, st);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    *converged = false;
    int round = 0;
    for (int sweep = 0; sweep < kMaxSweeps && !*converged; sweep++) {
        for (int r = 0; r < L.max_rounds; r++, round++) {
            e = prof_timed("dm_jacobi_pairs", stream, [&] {
                hipLaunchKernelGGL(dm_pair_kernel, dim3((unsigned)L.pair_items.size()), dim3(kPairThreads), 0, stream, secs,
                                   pair_items, A, Qw, (const DmState*)st, flags, round);
                return hipGetLastError();
            });
            if (e != hipSuccess) return e;
            e = prof_timed("dm_jacobi_update", stream, [&] {
                hipLaunchKernelGGL(dm_update_kernel, dim3((unsigned)L.upd_items.size()), dim3(256), 0, stream, secs,
                                   upd_items, A, Vw, (const double*)Qw, st, (const int*)flags, round);
                return hipGetLastError();
            });
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(dm_count_kernel, dim3(1), dim3(256), 0, stream, (const DmState*)st, n_sec, count);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        int host_count = -1;
        e = hipMemcpyAsync(&host_count, count, sizeof(int), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
        *converged = host_count == 0;
    }
    int64_t total = 0;
    for (int k = 0; k < n_sec; k++) total += sectors[k].n;
    return prof_timed("dm_sort_select", stream, [&] {
        hipLaunchKernelGGL(dm_sort_kernel, dim3(n_sec), dim3(256), 0, stream, secs, (const double*)A,
                           (const double*)Vw, W);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(dm_select_kernel, dim3(1), dim3(kSelThreads), 0, stream, secs, n_sec, (const double*)W, m_keep,
                           total, reinterpret_cast<int*>(ws + L.off_above), reinterpret_cast<int*>(ws + L.off_equal),
                           reinterpret_cast<double*>(ws + L.off_part), kept, eps);
        return hipGetLastError();
    });
}

}  // namespace rot
