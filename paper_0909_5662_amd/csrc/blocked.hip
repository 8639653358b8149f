// Quantum-number block-sparse rotation (Eq. (10) and the paragraph after it):
// block operators and the truncation matrix are block-sparse in the
// (N_up, N_dn) sectors; an operator with shift Delta maps old sector q to
// q + Delta.  For an output block (T <- Q), T = Q + Delta, with q_s = Q - qn(s):
//
//   stage 1 (per site state s):  X_s = O(q_s+Delta <- q_s) * U_Q[s rows]
//   stage 2:                     out(T <- Q) = U_T^T * [X_s stacked over s]
//
// The rows of U_T run over s and then over the old states of T - qn(s) =
// q_s + Delta, which are exactly the rows of X_s, so stage 2 is one GEMM with
// K = M_T.  Stacked rows whose operator block is absent are zero-filled (a
// stage-1 problem with K = 0).  All small GEMMs of all operators go through
// two grouped launches (grouped.hip).  The work-lists depend only on the
// block structure and the buffers, and are cached per signature.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "buffer_rsrc.h"
#include "pinned_lru.h"
#include "rot_internal.h"

namespace rot {
namespace {

// cached block structures kept beyond those pinned by graph capture
constexpr size_t kPlanCacheSize = 8;

struct QN {
    int u, d;
    bool operator<(const QN& o) const { return u != o.u ? u < o.u : d < o.d; }
};

struct Structure {
    std::map<QN, int> old_idx, new_idx;
    std::vector<int64_t> M;                     // rows of U_Q per new sector
    std::vector<std::vector<int64_t>> rowstart;  // [new k][s]; -1 if old sector absent
};

bool build_structure(const rot_blocked_problem* p, Structure* st, std::string* why) {
    char buf[256];
    auto bad = [&](const char* msg) {
        *why = msg;
        return false;
    };
    if (p->d <= 0 || !p->site_qn) return bad("d must be positive and site_qn non-null");
    if (p->n_old <= 0 || !p->old_sec || p->n_new <= 0 || !p->new_sec) return bad("empty or null sector tables");
    int64_t off = 0;
    for (int k = 0; k < p->n_old; k++) {
        const rot_sector& s = p->old_sec[k];
        if (s.dim <= 0 || s.offset != off) {
            snprintf(buf, sizeof buf, "old sector %d: dim must be > 0 and offset the prefix sum", k);
            *why = buf;
            return false;
        }
        off += s.dim;
        if (!st->old_idx.emplace(QN{s.n_up, s.n_dn}, k).second) return bad("duplicate old sector quantum numbers");
    }
    off = 0;
    for (int k = 0; k < p->n_new; k++) {
        const rot_sector& s = p->new_sec[k];
        if (s.dim <= 0 || s.offset != off) {
            snprintf(buf, sizeof buf, "kept sector %d: dim must be > 0 and offset the prefix sum", k);
            *why = buf;
            return false;
        }
        off += s.dim;
        if (!st->new_idx.emplace(QN{s.n_up, s.n_dn}, k).second) return bad("duplicate kept sector quantum numbers");
    }
    st->M.assign(p->n_new, 0);
    st->rowstart.assign(p->n_new, std::vector<int64_t>(p->d, -1));
    for (int k = 0; k < p->n_new; k++) {
        int64_t rows = 0;
        for (int s = 0; s < p->d; s++) {
            const QN q{p->new_sec[k].n_up - p->site_qn[2 * s], p->new_sec[k].n_dn - p->site_qn[2 * s + 1]};
            auto it = st->old_idx.find(q);
            if (it == st->old_idx.end()) continue;
            st->rowstart[k][s] = rows;
            rows += p->old_sec[it->second].dim;
        }
        if (rows < p->new_sec[k].dim) {
            snprintf(buf, sizeof buf, "kept sector %d has %d states but only %lld block-site states", k,
                     p->new_sec[k].dim, (long long)rows);
            *why = buf;
            return false;
        }
        st->M[k] = rows;
        if (!p->U_off || p->U_off[k] < 0) return bad("U_off missing or negative");
    }
    if (p->n_ops < 0) return bad("negative n_ops");
    if (p->n_ops > 0 && (!p->shift || !p->O_off || !p->out_off || !p->O_blk || !p->out_blk || !p->U_blk))
        return bad("null shift / O_off / out_off / O_blk / out_blk / U_blk");
    for (int b = 0; b < p->n_ops; b++) {
        const int du = p->shift[2 * b], dd = p->shift[2 * b + 1];
        for (int k = 0; k < p->n_new; k++) {
            if (p->out_off[(int64_t)b * p->n_new + k] < 0) continue;
            const QN t{p->new_sec[k].n_up + du, p->new_sec[k].n_dn + dd};
            if (!st->new_idx.count(t)) {
                snprintf(buf, sizeof buf, "operator %d: output block for kept sector %d requested but its target "
                         "sector (%d,%d) is not kept", b, k, t.u, t.d);
                *why = buf;
                return false;
            }
        }
        for (int k = 0; k < p->n_old; k++) {
            if (p->O_off[(int64_t)b * p->n_old + k] < -1) return bad("O_off entries must be >= -1");
        }
    }
    return true;
}

bool aligned16(const float* base, int64_t off) { return ((reinterpret_cast<uintptr_t>(base + off)) & 15) == 0; }

// ------------------------------------------------------------ fused path --
// One 64-wide wave per output block (operator b, kept sector Q), computing
//   Out^T(Q <- T) = sum_s X_s^T U_T[s rows],   X_s = O(q_s+Delta <- q_s) U_Q[s rows]
// on v_mfma_f32_16x16x4f32 (lane l supplies A(l%16, l/16), B(l/16, l%16);
// accumulator element v of lane l is D(4*(l/16)+v, l%16)).  A 16 x 16 block
// of X_s in accumulator layout is, read with the k order 4*(l/16)+j at step
// j, exactly the A operand of X_s^T: X never leaves registers.  Stage 1 uses
// the same k order (16-wide k groups, lane group h taking k = 4h + j at step
// j), so every lane fetches four consecutive k with one 16-byte load in both
// stages.  For that the U blocks are read transposed from the workspace
// (U^T_Q[beta][padded row], filled per call by transpose_u_kernel): each
// site state's rows start at a multiple of 4 and the padding is zero.
struct BlkTask {
    int mT, mQ;          // output block rows (kept dim of T) and columns (kept dim of Q)
    int term0, n_terms;  // terms (site states with a non-zero operator block)
    int ldT, ldQ;        // padded row counts of U^T_T and U^T_Q (leading dimensions)
    int64_t uT_off;      // U^T_T in the transposed-U area
    int64_t uQ_off;      // U^T_Q in the transposed-U area
    int64_t out_off;     // output block in out_blk, leading dimension mQ
};
struct BlkTerm {
    int a, k;        // rows of X_s (old states of q_s + Delta), stage-1 K (old states of q_s)
    int rt, rq;      // first padded row of site state s in U^T_T and in U^T_Q (multiples of 4)
    int64_t o_off;   // operator block (a x k, leading dimension k) in O_blk
};
// One site state's rows of one kept sector in the transposed-U area.  With
// rows = 0 it writes zeros instead: mp runs of rows4 zeros, ld apart (the
// alignment gaps and the slack of the area; the Xt segments of site states
// whose source sector is absent, one run per operator).
struct UtSeg {
    int64_t u_off;   // first row of the segment in U_blk (leading dimension mp)
    int64_t ut_off;  // workspace offset (floats) of column 0 of this segment (leading dimension ld)
    int rows, rows4, mp, ld;
};

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));

// Slack after the transposed-U area: stage 1 reads up to CG - 1 column
// blocks (and a partial one) past a sector, i.e. fewer than 96 rows of the
// widest block, and padded k runs past a row by fewer than 16 values.  The
// transpose writes the whole area (zeros in the padding rows, the alignment
// gaps between sectors and the slack), so such reads only meet finite values.
inline int64_t ut_slack(int max_ld) { return 96 * (int64_t)max_ld + 64; }

__global__ __launch_bounds__(256) void transpose_u_kernel(const UtSeg* __restrict__ segs, const float* __restrict__ U,
                                                          float* __restrict__ Ut) {
    const UtSeg g = segs[blockIdx.y];
    const int64_t n = (int64_t)g.rows4 * g.mp;
    if (g.rows == 0) {  // zero runs, each written contiguously
        for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
            Ut[g.ut_off + (e / g.rows4) * g.ld + e % g.rows4] = 0.f;
        return;
    }
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int i = (int)(e / g.mp), beta = (int)(e % g.mp);
        Ut[g.ut_off + (int64_t)beta * g.ld + i] = i < g.rows ? U[g.u_off + (int64_t)i * g.mp + beta] : 0.f;
    }
}

// Four consecutive floats at row + kk when `full`, else zero.  The address
// falls back to `safe` (a readable 16-byte location) so that the load is
// unconditional and the choice a select, not a branch.
template <bool VEC>
__device__ __forceinline__ f32x4 quad_or_zero(const float* row, int kk, bool full, const float* safe) {
    const float* a = full ? row + kk : safe;
    const f32x4 v = VEC ? *reinterpret_cast<const f32x4*>(a) : *reinterpret_cast<const f32x4u*>(a);
    return full ? v : f32x4{0.f, 0.f, 0.f, 0.f};
}

// MAXA: most 16-wide blocks of output rows (kept dim of T) a task can have;
// CG: output column blocks (kept dim of Q) handled together, so each value of
// the operator block fetched in stage 1 feeds CG instructions and each value
// of U_T fetched in stage 2 feeds CG instructions.
template <int MAXA, int CG>
__global__ __launch_bounds__(256) void blocked_fused_kernel(const BlkTask* __restrict__ tasks, int n_tasks,
                                                            const BlkTerm* __restrict__ terms,
                                                            const float* __restrict__ Ut, const float* __restrict__ O,
                                                            float* __restrict__ out, int* __restrict__ counter) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lh = lane >> 4;
    int t = 0;
    if (lane == 0) t = atomicAdd(counter, 1);
    t = __builtin_amdgcn_readfirstlane(t);  // lane 0's ticket, uniform over the wave
    while (t < n_tasks) {
        const BlkTask T = tasks[t];
        const float* uT = Ut + T.uT_off;
        const float* uQ = Ut + T.uQ_off;
        const int nbc = (T.mQ + 15) >> 4, nba = (T.mT + 15) >> 4;
        for (int cg0 = 0; cg0 < nbc; cg0 += CG) {
            f32x4 acc[CG][MAXA];
#pragma unroll
            for (int c = 0; c < CG; c++)
#pragma unroll
                for (int ca = 0; ca < MAXA; ca++) acc[c][ca] = f32x4{0.f, 0.f, 0.f, 0.f};
            for (int e = 0; e < T.n_terms; e++) {
                const BlkTerm tm = terms[T.term0 + e];
                const float* o = O + tm.o_off;
                for (int rb = 0; rb * 16 < tm.a; rb++) {
                    // stage 2's U_T values for this row block do not depend on
                    // stage 1: their loads are issued first and overlap it
                    f32x4 ut[MAXA];
#pragma unroll
                    for (int ca = 0; ca < MAXA; ca++)
                        if (ca < nba)
                            ut[ca] = *reinterpret_cast<const f32x4*>(uT + (int64_t)(ca * 16 + li) * T.ldT + tm.rt +
                                                                     rb * 16 + 4 * lh);
                    // stage 1: X_s rows 16 rb.., column blocks cg0 .. cg0+CG-1;
                    // the operands of the next 16 k load while this step multiplies
                    f32x4 x[CG];
#pragma unroll
                    for (int c = 0; c < CG; c++) x[c] = f32x4{0.f, 0.f, 0.f, 0.f};
                    const int row = rb * 16 + li;
                    const bool rok = row < tm.a;
                    const float* orow = o + (int64_t)row * tm.k;
                    auto load_a = [&](int k0) __attribute__((always_inline)) {
                        const int kk = k0 + 4 * lh;  // this lane's k = kk + j at step j
                        f32x4 av = quad_or_zero<false>(orow, kk, rok && kk + 4 <= tm.k, Ut);
                        if ((tm.k & 3) != 0 && rok && kk < tm.k && kk + 4 > tm.k) {
                            // the row's last, partial quad
#pragma unroll
                            for (int j = 0; j < 4; j++) av[j] = kk + j < tm.k ? orow[kk + j] : 0.f;
                        }
                        return av;
                    };
                    f32x4 av = f32x4{0.f, 0.f, 0.f, 0.f}, bv[CG];
#pragma unroll
                    for (int c = 0; c < CG; c++) bv[c] = av;
                    if (tm.k > 0) {
                        av = load_a(0);
#pragma unroll
                        for (int c = 0; c < CG; c++)
                            bv[c] = *reinterpret_cast<const f32x4*>(uQ + (int64_t)((cg0 + c) * 16 + li) * T.ldQ +
                                                                    tm.rq + 4 * lh);
                    }
                    for (int k0 = 0; k0 < tm.k; k0 += 16) {
                        f32x4 av_n = av, bv_n[CG];
#pragma unroll
                        for (int c = 0; c < CG; c++) bv_n[c] = bv[c];
                        if (k0 + 16 < tm.k) {
                            av_n = load_a(k0 + 16);
#pragma unroll
                            for (int c = 0; c < CG; c++)
                                bv_n[c] = *reinterpret_cast<const f32x4*>(
                                    uQ + (int64_t)((cg0 + c) * 16 + li) * T.ldQ + tm.rq + k0 + 16 + 4 * lh);
                        }
#pragma unroll
                        for (int j = 0; j < 4; j++)
#pragma unroll
                            for (int c = 0; c < CG; c++)
                                x[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[j], bv[c][j], x[c], 0, 0, 0);
                        av = av_n;
#pragma unroll
                        for (int c = 0; c < CG; c++) bv[c] = bv_n[c];
                    }
                    // stage 2: acc(beta, alpha) += sum_r X_s[r][beta] U_T[rt + r][alpha], the X block
                    // in accumulator layout read with k order 4*(l/16) + j at step j
#pragma unroll
                    for (int ca = 0; ca < MAXA; ca++) {
                        if (ca < nba) {
#pragma unroll
                            for (int j = 0; j < 4; j++)
#pragma unroll
                                for (int c = 0; c < CG; c++)
                                    acc[c][ca] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[c][j], ut[ca][j], acc[c][ca], 0,
                                                                                       0, 0);
                        }
                    }
                }
            }
            // acc[c][ca] element v of lane l = Out^T(beta = 16 (cg0+c) + 4*(l/16) + v, alpha = 16 ca + l%16)
#pragma unroll
            for (int c = 0; c < CG; c++)
#pragma unroll
                for (int ca = 0; ca < MAXA; ca++) {
                    const int alpha = ca * 16 + li;
                    if (ca < nba && alpha < T.mT) {
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            const int b = (cg0 + c) * 16 + 4 * lh + v;
                            if (b < T.mQ) out[T.out_off + (int64_t)alpha * T.mQ + b] = acc[c][ca][v];
                        }
                    }
                }
        }
        if (lane == 0) t = atomicAdd(counter, 1);
        t = __builtin_amdgcn_readfirstlane(t);  // lane 0's ticket, uniform over the wave
    }
}

// Variant of blocked_fused_kernel that loads the operator rows of a whole
// (term, row block) pair at once (every k step's rows requested together),
// and requests the next pair's rows while the current pair multiplies: the
// operator blocks come from HBM, and the wave then waits for an HBM round
// trip only at the first pair of a pass.  U^T_Q values (L2-resident) are
// fetched one k step ahead.  Needs every term's stage-1 K <= 16 * KS.
template <int MAXA, int CG, int KS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void blocked_rowblock_kernel(const BlkTask* __restrict__ tasks, int n_tasks,
                                                               const BlkTerm* __restrict__ terms,
                                                               const float* __restrict__ Ut,
                                                               const float* __restrict__ O, float* __restrict__ out,
                                                               int* __restrict__ counter) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lh = lane >> 4;
    // the operator rows of row block rb of term tm, every k step (zero past
    // the block)
    auto load_rows = [&](const BlkTerm& tm, int rb, f32x4* a) __attribute__((always_inline)) {
        const int nks = (tm.k + 15) >> 4;
        const int row = rb * 16 + li;
        const bool rok = row < tm.a;
        const float* orow = O + tm.o_off + (int64_t)(rok ? row : 0) * tm.k;
#pragma unroll
        for (int ks = 0; ks < KS; ks++) {
            const int kk = ks * 16 + 4 * lh;
            if (ks < nks) a[ks] = quad_or_zero<false>(orow, kk, rok && kk + 4 <= tm.k, Ut);
        }
        // the row's last, partial quad (K not a multiple of 4)
        const int kt = 16 * (nks - 1) + 4 * lh;
        if ((tm.k & 3) != 0 && rok && kt < tm.k && kt + 4 > tm.k) {
#pragma unroll
            for (int ks = 0; ks < KS; ks++)
                if (ks == nks - 1) {
#pragma unroll
                    for (int j = 0; j < 4; j++) a[ks][j] = kt + j < tm.k ? orow[kt + j] : 0.f;
                }
        }
    };
    int t = 0;
    if (lane == 0) t = atomicAdd(counter, 1);
    t = __builtin_amdgcn_readfirstlane(t);
    while (t < n_tasks) {
        const BlkTask T = tasks[t];
        const float* uT = Ut + T.uT_off;
        const float* uQ = Ut + T.uQ_off;
        const int nbc = (T.mQ + 15) >> 4, nba = (T.mT + 15) >> 4;
        for (int cg0 = 0; cg0 < nbc; cg0 += CG) {
            f32x4 acc[CG][MAXA];
#pragma unroll
            for (int c = 0; c < CG; c++)
#pragma unroll
                for (int ca = 0; ca < MAXA; ca++) acc[c][ca] = f32x4{0.f, 0.f, 0.f, 0.f};
            // walk the (term, row block) pairs of the task in order
            int e = 0, rb = 0;
            BlkTerm tm{};
            f32x4 a[KS];
            if (T.n_terms > 0) {
                tm = terms[T.term0];
                load_rows(tm, 0, a);
            }
            while (e < T.n_terms) {
                // the pair after this one
                int e2 = e, rb2 = rb + 1;
                BlkTerm tm2 = tm;
                if (rb2 * 16 >= tm.a) {
                    e2 = e + 1;
                    rb2 = 0;
                    if (e2 < T.n_terms) tm2 = terms[T.term0 + e2];
                }
                const int nks = (tm.k + 15) >> 4;
                f32x4 ut[MAXA];
#pragma unroll
                for (int ca = 0; ca < MAXA; ca++)
                    if (ca < nba)
                        ut[ca] = *reinterpret_cast<const f32x4*>(uT + (int64_t)(ca * 16 + li) * T.ldT + tm.rt +
                                                                 rb * 16 + 4 * lh);
                f32x4 x[CG], bv[CG];
#pragma unroll
                for (int c = 0; c < CG; c++) x[c] = f32x4{0.f, 0.f, 0.f, 0.f};
                if (nks > 0) {
#pragma unroll
                    for (int c = 0; c < CG; c++)
                        bv[c] = *reinterpret_cast<const f32x4*>(uQ + (int64_t)((cg0 + c) * 16 + li) * T.ldQ + tm.rq +
                                                                4 * lh);
                }
                // the next pair's operator rows load while this pair multiplies
                f32x4 an[KS];
                if (e2 < T.n_terms) load_rows(tm2, rb2, an);
#pragma unroll
                for (int ks = 0; ks < KS; ks++) {
                    if (ks < nks) {
                        f32x4 bv_n[CG];
                        if (ks + 1 < nks) {
#pragma unroll
                            for (int c = 0; c < CG; c++)
                                bv_n[c] = *reinterpret_cast<const f32x4*>(
                                    uQ + (int64_t)((cg0 + c) * 16 + li) * T.ldQ + tm.rq + (ks + 1) * 16 + 4 * lh);
                        }
#pragma unroll
                        for (int j = 0; j < 4; j++)
#pragma unroll
                            for (int c = 0; c < CG; c++)
                                x[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ks][j], bv[c][j], x[c], 0, 0, 0);
                        if (ks + 1 < nks) {
#pragma unroll
                            for (int c = 0; c < CG; c++) bv[c] = bv_n[c];
                        }
                    }
                }
                // stage 2 (as in blocked_fused_kernel)
#pragma unroll
                for (int ca = 0; ca < MAXA; ca++) {
                    if (ca < nba) {
#pragma unroll
                        for (int j = 0; j < 4; j++)
#pragma unroll
                            for (int c = 0; c < CG; c++)
                                acc[c][ca] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[c][j], ut[ca][j], acc[c][ca], 0,
                                                                                   0, 0);
                    }
                }
                e = e2;
                rb = rb2;
                tm = tm2;
#pragma unroll
                for (int ks = 0; ks < KS; ks++) a[ks] = an[ks];
            }
#pragma unroll
            for (int c = 0; c < CG; c++)
#pragma unroll
                for (int ca = 0; ca < MAXA; ca++) {
                    const int alpha = ca * 16 + li;
                    if (ca < nba && alpha < T.mT) {
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            const int b = (cg0 + c) * 16 + 4 * lh + v;
                            if (b < T.mQ) out[T.out_off + (int64_t)alpha * T.mQ + b] = acc[c][ca][v];
                        }
                    }
                }
        }
        if (lane == 0) t = atomicAdd(counter, 1);
        t = __builtin_amdgcn_readfirstlane(t);
    }
}

// ---------------------------------------------------------- stacked path --
// Operators with the same shift Delta share every block of U, so each
// stage's small products over all of them form one GEMM per sector
// combination, with the operators stacked along N:
//   stage 1, per (Delta, source sector q), for each site state s with
//   Q = q + qn(s):
//     Xt_b(Q)[beta][r_s + i] = sum_k U_Q[s rows][k][beta] O_b(q+Delta <- q)[i][k]
//   stage 2, per (Delta, Q), T = Q + Delta:
//     out_b(T <- Q)[alpha][beta] = sum_r U_T[r][alpha] Xt_b(Q)[beta][r]
// Both are C[m][n] = sum_k A[m][k] B[n][k]: A is a row of the transposed-U
// area shared by the group, B and C rows belong to operator j = n / nb.  The
// 16-wide instruction tiles then pad only one extent per stage (M, a kept
// sector dimension) instead of all three.  Xt_b(Q) (m'_Q rows over the padded
// rows r of U^T_T) lives in the workspace stored segment by segment: site
// state s's columns [r_s, r_s + a4) form an m'_Q x a4 row-major block, so a
// stage-1 tile writes whole cache lines; padding columns are written as zeros.
struct StkGroup {
    int M, N, K;    // C is M x N, contraction length K
    int nb;         // columns per operator: n = j nb + i
    int nvalid;     // B rows with i >= nvalid are zero
    int lda, ldb;   // A row stride; B row stride inside an operator block
    int ldcm;       // C stride per row m (stage 2: m'_Q; streamed stage 1: the segment width)
    int64_t a_off;  // A row 0 in the transposed-U area
    int64_t tab;    // first entry of the group in the per-operator tables
    // stage 2 reads Xt blocks stored segment by segment: k in [seg[s],
    // seg[s + 1]) is column k - seg[s] of an nb x (seg[s + 1] - seg[s])
    // row-major block at nb * seg[s]; unused entries hold kSegEnd
    int seg[5];
    int pad;
};
struct StkTile {
    int group, m0, n0, pad;
};
constexpr int kStkMB = 5;  // 16-row blocks per wave tile (80 rows)
constexpr int kSegEnd = 1 << 30;
constexpr int kStkNB = 4;  // 16-column blocks per wave tile (64 columns)

// One wave per tile part (a 16 NB-column share of a 64-column tile), four
// waves per workgroup.  boff[tab + j] locates operator j's B block (-1:
// absent, zero rows), coff[tab + j] its C block (-1: not written).  PF: 16-wide k steps whose
// loads are in flight while a step multiplies.  BVEC: B rows are 16-byte
// aligned (stage 2); otherwise only 4-byte aligned.
template <int NB, int PF, bool BVEC, bool SEG>
__global__ __launch_bounds__(256) void blocked_stacked_kernel(const StkTile* __restrict__ tiles, int n_tiles,
                                                              const StkGroup* __restrict__ groups,
                                                              const int64_t* __restrict__ boff,
                                                              const int64_t* __restrict__ coff,
                                                              const float* __restrict__ A,
                                                              const float* __restrict__ B, float* __restrict__ C) {
    constexpr int MB = kStkMB;
    constexpr int PARTS = kStkNB / NB;
    static_assert(kStkNB % NB == 0, "whole column parts");
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lh = lane >> 4;
    const int w = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int t = w / PARTS;
    if (t >= n_tiles) return;
    const StkTile tl = tiles[t];
    const StkGroup g = groups[tl.group];
    const int n0 = tl.n0 + (w % PARTS) * 16 * NB;
    if (n0 >= g.N) return;
    const int nbm = min(MB, (g.M - tl.m0 + 15) >> 4);
    const int nbn = min(NB, (g.N - n0 + 15) >> 4);
    // this lane's A row in each row block and B / C row in each column block
    const float* arow[MB];
    bool aok[MB];
#pragma unroll
    for (int mb = 0; mb < MB; mb++) {
        const int m = tl.m0 + mb * 16 + li;
        aok[mb] = m < g.M;
        arow[mb] = A + g.a_off + (int64_t)(aok[mb] ? m : 0) * g.lda;
    }
    const float* brow[NB];
    float* crow[NB];
    bool bok[NB], cok[NB];
    int brw[NB];  // SEG: this lane's row of the operator's Xt block
#pragma unroll
    for (int nb = 0; nb < NB; nb++) {
        const int n = n0 + nb * 16 + li;
        cok[nb] = n < g.N;
        const int j = cok[nb] ? n / g.nb : 0;
        const int i = n - j * g.nb;
        brw[nb] = i;
        const int64_t bo = cok[nb] ? boff[g.tab + j] : -1;
        bok[nb] = cok[nb] && i < g.nvalid && bo >= 0;
        brow[nb] = B + (bok[nb] ? bo + (SEG ? 0 : (int64_t)i * g.ldb) : 0);
        const int64_t co = cok[nb] ? coff[g.tab + j] : -1;
        cok[nb] = co >= 0;  // no output block: nothing to write
        crow[nb] = C + (cok[nb] ? co + i : 0);
    }
    const int K = g.K;
    const int nks = (K + 15) >> 4;
    struct Ops {
        f32x4 a[MB], b[NB];
    };
    // lane group lh takes k = 16 s + 4 lh + q at instruction q of step s.  A
    // rows (the transposed-U area) are zero-padded to a multiple of 4, so a
    // quad starting below K is whole; B rows end at K: a quad crossing K (K
    // not a multiple of 4, last step only) is read element by element.
    auto fetch = [&](Ops& o, int s) __attribute__((always_inline)) {
        const int kk = 16 * s + 4 * lh;
#pragma unroll
        for (int mb = 0; mb < MB; mb++)
            if (mb < nbm) o.a[mb] = quad_or_zero<true>(arow[mb], kk, aok[mb] && kk < K, A);
        if (SEG) {
            // the segment holding k = kk .. kk + 3 (segments are multiples of 4 wide)
            const int sg = (kk >= g.seg[1]) + (kk >= g.seg[2]) + (kk >= g.seg[3]);
            const int p0 = sg == 0 ? 0 : sg == 1 ? g.seg[1] : sg == 2 ? g.seg[2] : g.seg[3];
            const int p1 = sg == 0 ? g.seg[1] : sg == 1 ? g.seg[2] : sg == 2 ? g.seg[3] : g.seg[4];
            const int64_t off = (int64_t)g.nb * p0 - p0;
#pragma unroll
            for (int nb = 0; nb < NB; nb++)
                if (nb < nbn)
                    o.b[nb] = quad_or_zero<BVEC>(brow[nb] + off + (int64_t)brw[nb] * (p1 - p0), kk,
                                                 bok[nb] && kk < K, A);
        } else {
#pragma unroll
            for (int nb = 0; nb < NB; nb++)
                if (nb < nbn) o.b[nb] = quad_or_zero<BVEC>(brow[nb], kk, bok[nb] && kk + 4 <= K, A);
        }
        if (!SEG && (K & 3) != 0 && s == nks - 1 && kk < K && kk + 4 > K) {
#pragma unroll
            for (int nb = 0; nb < NB; nb++)
                if (nb < nbn && bok[nb]) {
#pragma unroll
                    for (int q = 0; q < 4; q++) o.b[nb][q] = kk + q < K ? brow[nb][kk + q] : 0.f;
                }
        }
    };
    f32x4 acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; mb++)
#pragma unroll
        for (int nb = 0; nb < NB; nb++) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    auto multiply = [&](const Ops& o) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
            for (int mb = 0; mb < MB; mb++)
#pragma unroll
                for (int nb = 0; nb < NB; nb++)
                    if (mb < nbm && nb < nbn)
                        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(o.a[mb][q], o.b[nb][q], acc[mb][nb], 0, 0, 0);
    };
    // step s multiplies `cur` after issuing the loads of step s + PF into `dst`
    auto step = [&](int s, const Ops& cur, Ops& dst) __attribute__((always_inline)) {
        if (s + PF < nks) fetch(dst, s + PF);
        multiply(cur);
    };
    // ring of PF + 1 operand sets, unrolled so every set is a fixed register set
    Ops o[PF + 1];
#pragma unroll
    for (int s = 0; s < PF; s++)
        if (s < nks) fetch(o[s], s);
    for (int s0 = 0; s0 < nks; s0 += PF + 1) {
#pragma unroll
        for (int r = 0; r <= PF; r++)
            if (s0 + r < nks) step(s0 + r, o[r], o[(r + PF) % (PF + 1)]);
    }
    // accumulator element v of lane l: C(m0 + 16 mb + 4 (l / 16) + v, column l % 16 of block nb)
#pragma unroll
    for (int mb = 0; mb < MB; mb++)
#pragma unroll
        for (int nb = 0; nb < NB; nb++)
            if (mb < nbm && nb < nbn && cok[nb]) {
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int m = tl.m0 + mb * 16 + 4 * lh + v;
                    if (m < g.M) crow[nb][(int64_t)m * g.ldcm] = acc[mb][nb][v];
                }
            }
}

// Stage 1 for source sectors of at most 80 states: one group per (shift,
// source sector q) stacks the operators' blocks O(q + Delta <- q) along N;
// its members are the U^T_Q rows of each site state s whose kept sector
// Q = q + qn(s) has output blocks (row tiles of at most 80).  One workgroup
// takes 64 stacked columns and up to four members: the 64 operator rows
// (every k) are staged once in LDS and shared by its eight waves, two per
// member on 32 columns each, which multiply them by the member's U^T rows
// (fetched one k step ahead) and store their tiles as their last memory
// operation.  Each member tile writes one Xt segment (m'_Q x a4 row-major,
// a4 the source block's row count rounded up to 4) as a dense block.
struct StkMember {
    int M;           // rows of this member tile (<= 80)
    int lda, ldcm;   // A row stride; C stride per row (the segment width a4)
    int span;        // bytes of the Xt group of the member's (shift, Q), at most kStkSpanMax
    int64_t a_off;   // A row 0 in the transposed-U area
    int64_t tab;     // per-operator C offsets into Xt (-1: operator has no output block)
    int64_t c_base;  // first element of that Xt group: the stores address it through a buffer descriptor
};
// Stage-1 store offsets (bytes, 32-bit) into one Xt group of at most
// kStkSpanMax bytes; the hardware drops a store at or past the group's end.
// An operator without an output block starts its rows at kStkNoBlock (rows
// add less than 2^16), a row past M stores at kStkDrop.
constexpr int kStkSpanMax = 0x3fffffc0;
constexpr int kStkNoBlock = 0x40000000;
constexpr int kStkDrop = 0x7ffffff0;
struct StkGroupR {
    int N, K, nb, nvalid;  // C columns, contraction length, columns per operator, non-zero rows of each
    int pad0, pad1;
    int64_t tab;  // per-operator B offsets into O_blk (-1: block absent)
};
constexpr int kStkResK = 5;  // 16-wide k steps staged (K <= 80)

// tiles[blockIdx.x] = {group, first member, first stacked column, members};
// eight waves: two per member, each on 32 of the columns.
template <int PFA>
__global__ __launch_bounds__(512) void blocked_stacked_lds_kernel(const StkTile* __restrict__ tiles,
                                                                        const StkGroupR* __restrict__ groups,
                                                                        const StkMember* __restrict__ members,
                                                                        const int64_t* __restrict__ boff,
                                                                        const int64_t* __restrict__ coff,
                                                                        const float* __restrict__ A,
                                                                        const float* __restrict__ B,
                                                                        float* __restrict__ C, int abytes) {
    constexpr int WPM = 2;  // waves per member
    constexpr int MB = kStkMB, NB = kStkNB / WPM, KS = kStkResK, ROWS = 16 * kStkNB, NT = 256 * WPM;
    __shared__ f32x4 bs[4 * KS][ROWS];  // operator rows: [k quad][stacked column], 20 KiB
    // per wave: one 16-row block of its 16 x 32 output tile, transposed so
    // that each lane stores four consecutive columns (row pitch 36: the four
    // lane groups of a write fall in different banks), 18 KiB
    constexpr int TP = 36;
    __shared__ __attribute__((aligned(16))) float tt[NT / 64][16 * TP];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int li = lane & 15, lh = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = w / WPM;                 // member of this wave
    const int c0 = (w % WPM) * 16 * NB;     // its first column in the tile
    const StkTile tl = tiles[blockIdx.x];
    const StkGroupR g = groups[tl.group];
    const int K = g.K;
    const int nks = (K + 15) >> 4;
    const int n0 = tl.n0 + c0;
    const int nbn = max(0, min(NB, (g.N - n0 + 15) >> 4));
    // this wave's member: its U^T rows, output rows, first k step
    const bool active = wm < tl.pad && nbn > 0;
    StkMember mem{};
    if (active) mem = members[tl.m0 + wm];
    const int nbm = min(MB, (mem.M + 15) >> 4);
    // U^T rows through a descriptor over the transposed-U area (abytes <
    // 2^30) at 32-bit byte offsets; a row past M, or a quad at or past K,
    // reads at kStkDrop, past the end, and gets zeros
    const __amdgpu_buffer_rsrc_t ares =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(A), (short)0, abytes, kBufferFlags);
    int aofs[MB];
#pragma unroll
    for (int mb = 0; mb < MB; mb++) {
        const int m = mb * 16 + li;
        aofs[mb] = active && m < mem.M ? (int)((mem.a_off + (int64_t)m * mem.lda) * 4) : kStkDrop;
    }
    auto aquad = [&](int mb, int kk) __attribute__((always_inline)) {
        const int off = kk < K && aofs[mb] != kStkDrop ? aofs[mb] + 4 * kk : kStkDrop;
        return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ares, off, 0, 0));
    };
    // U^T rows of k steps s .. s + PFA in flight: set s % (PFA + 1) holds step s
    f32x4 a[PFA + 1][MB];
#pragma unroll
    for (int p = 0; p < PFA; p++)
        if (p < nks) {
#pragma unroll
            for (int mb = 0; mb < MB; mb++)
                if (mb < nbm) {
                    a[p][mb] = aquad(mb, 16 * p + 4 * lh);
                }
        }
    // stores: 32-bit byte offsets into the member's Xt group; an operator
    // without an output block, or a row past M, gets an offset past the group
    // instead of a branch, and the hardware drops that store
    const __amdgpu_buffer_rsrc_t cres =
        __builtin_amdgcn_make_buffer_rsrc(C + mem.c_base, (short)0, mem.span, kBufferFlags);
    const int ldc4 = mem.ldcm * 4;  // bytes from one Xt row to the next
    // this lane's stores: columns 4 (lane % 8) .. + 3 of the wave's 32 (one
    // operator's: segments are multiples of 4 wide), rows lane / 8 and
    // lane / 8 + 8 of each 16-row block
    const int sq = lane & 7, sr = lane >> 3;
    int qofs;
    {
        const int n = n0 + 4 * sq;
        const bool ok = active && n < g.N;
        const int j = ok ? n / g.nb : 0;
        const int64_t co = ok ? coff[mem.tab + j] : -1;
        qofs = (co >= 0 ? (int)((co - mem.c_base + (n - j * g.nb)) * 4) : kStkNoBlock) + sr * ldc4;
    }
    const int mrem8 = mem.M - sr;  // rows mb * 16 + 8 h of this lane exist while below this
    // stage the operator rows: thread tid owns stacked column tid % 64 and
    // k quads tid / 64 + (NT / 64) i (zero past K; a quad crossing K element
    // by element)
    {
        const int r = tid & (ROWS - 1);
        const int n = tl.n0 + r;
        const bool ok = n < g.N;
        const int j = ok ? n / g.nb : 0;
        const int i = n - j * g.nb;
        const int64_t bo = ok ? boff[g.tab + j] : -1;
        const bool bok = ok && i < g.nvalid && bo >= 0;
        const float* brow = B + (bok ? bo + (int64_t)i * K : 0);
#pragma unroll
        for (int x = 0; x < (4 * KS * ROWS + NT - 1) / NT; x++) {
            const int kq = w + (NT / 64) * x;
            if (kq < 4 * nks) {
                const int kk = 4 * kq;
                f32x4 v = quad_or_zero<false>(brow, kk, bok && kk + 4 <= K, A);
                if ((K & 3) != 0 && bok && kk < K && kk + 4 > K) {
#pragma unroll
                    for (int q = 0; q < 4; q++) v[q] = kk + q < K ? brow[kk + q] : 0.f;
                }
                bs[kq][r] = v;
            }
        }
    }
    __syncthreads();
    if (!active) return;
    // the member's row-block count as a compile-time constant, so the
    // products and stores carry no per-instruction guards (a column past N
    // multiplies the zeros staged for it and is not stored)
    auto run = [&](auto nbm_c) __attribute__((always_inline)) {
        constexpr int NBM = decltype(nbm_c)::value;
        f32x4 acc[NBM][NB];
#pragma unroll
        for (int mb = 0; mb < NBM; mb++)
#pragma unroll
            for (int nb = 0; nb < NB; nb++) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < KS; s++) {
            if (s < nks) {
                if (s + PFA < nks) {
#pragma unroll
                    for (int mb = 0; mb < NBM; mb++) {
                        a[(s + PFA) % (PFA + 1)][mb] = aquad(mb, 16 * (s + PFA) + 4 * lh);
                    }
                }
                // lane group lh takes k = 16 s + 4 lh + q at instruction q
                f32x4 bf[NB];
#pragma unroll
                for (int nb = 0; nb < NB; nb++) bf[nb] = bs[4 * s + lh][c0 + nb * 16 + li];
#pragma unroll
                for (int q = 0; q < 4; q++)
#pragma unroll
                    for (int mb = 0; mb < NBM; mb++)
#pragma unroll
                        for (int nb = 0; nb < NB; nb++)
                            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s % (PFA + 1)][mb][q], bf[nb][q],
                                                                               acc[mb][nb], 0, 0, 0);
            }
        }
        float* tw = tt[w];
#pragma unroll
        for (int mb = 0; mb < NBM; mb++) {
            // accumulator element v of lane l: row 4 (l / 16) + v, column nb * 16 + l % 16
#pragma unroll
            for (int nb = 0; nb < NB; nb++)
#pragma unroll
                for (int v = 0; v < 4; v++) tw[(4 * lh + v) * TP + nb * 16 + li] = acc[mb][nb][v];
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const int r = mb * 16 + 8 * h;
                const f32x4 q = *reinterpret_cast<const f32x4*>(tw + (sr + 8 * h) * TP + 4 * sq);
                const int off = r < mrem8 ? qofs + r * ldc4 : kStkDrop;
                __builtin_amdgcn_raw_buffer_store_b128(
                    u32x4{__float_as_uint(q[0]), __float_as_uint(q[1]), __float_as_uint(q[2]), __float_as_uint(q[3])},
                    cres, off, 0, 0);
            }
            __builtin_amdgcn_wave_barrier();
        }
    };
    static_assert(MB == 5, "one case per row-block count");
    switch (nbm) {
        case 1: run(std::integral_constant<int, 1>{}); break;
        case 2: run(std::integral_constant<int, 2>{}); break;
        case 3: run(std::integral_constant<int, 3>{}); break;
        case 4: run(std::integral_constant<int, 4>{}); break;
        case 5: run(std::integral_constant<int, 5>{}); break;
        default: break;
    }
}

// Stage 2 with U^T_T staged in LDS: one workgroup per (group, 80-row tile,
// 128 stacked columns), four waves of 32 columns.  Each 16-wide k step of the
// 80 A rows is fetched once for the four waves into one of two LDS buffers
// while the other is multiplied; the waves' own B rows (Xt, read segment by
// segment) stream through registers two k steps ahead.
constexpr int kStk2Cols = 128;  // stacked columns per workgroup
__global__ __launch_bounds__(256) void blocked_stacked2_wg_kernel(const StkTile* __restrict__ tiles,
                                                                  const StkGroup* __restrict__ groups,
                                                                  const int64_t* __restrict__ boff,
                                                                  const int64_t* __restrict__ coff,
                                                                  const float* __restrict__ A,
                                                                  const float* __restrict__ B, float* __restrict__ C,
                                                                  int abytes) {
    constexpr int MB = kStkMB, NB = 2, PF = 2, AR = 16 * kStkMB;
    __shared__ f32x4 as[2][4][AR];  // [buffer][k quad][row], 10 KiB
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int li = lane & 15, lh = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const StkTile tl = tiles[blockIdx.x];
    const StkGroup g = groups[tl.group];
    const int K = g.K;
    const int nks = (K + 15) >> 4;
    const int nbm = min(MB, (g.M - tl.m0 + 15) >> 4);
    const int n0 = tl.n0 + w * 16 * NB;
    const int nbn = max(0, min(NB, (g.N - n0 + 15) >> 4));
    // A staging: thread tid carries quads tid and tid + 256 of the 4 x 80 of
    // a step, read through a descriptor over the transposed-U area (abytes <
    // 2^30) at 32-bit byte offsets; a row past M or a quad at or past K reads
    // at kStkDrop, past the end, and gets zeros
    const __amdgpu_buffer_rsrc_t ares =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(A), (short)0, abytes, kBufferFlags);
    int aofs[2];
    bool aq[2];
    int akq[2], arw[2];
#pragma unroll
    for (int x = 0; x < 2; x++) {
        const int q = tid + 256 * x;
        aq[x] = q < 4 * AR;
        arw[x] = q % AR;
        akq[x] = q / AR;
        const int m = tl.m0 + arw[x];
        aofs[x] = aq[x] && m < g.M ? (int)((g.a_off + (int64_t)m * g.lda) * 4) : kStkDrop;
    }
    auto stage_load = [&](int s, f32x4* v) __attribute__((always_inline)) {
#pragma unroll
        for (int x = 0; x < 2; x++) {
            const int kk = 16 * s + 4 * akq[x];
            const int off = kk < K && aofs[x] != kStkDrop ? aofs[x] + 4 * kk : kStkDrop;
            v[x] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ares, off, 0, 0));
        }
    };
    auto stage_store = [&](int buf, const f32x4* v) __attribute__((always_inline)) {
#pragma unroll
        for (int x = 0; x < 2; x++)
            if (aq[x]) as[buf][akq[x]][arw[x]] = v[x];
    };
    // this wave's B rows: row brw of operator j's Xt block
    const float* brow[NB];
    float* crow[NB];
    bool bok[NB], cok[NB];
    int brw[NB];
#pragma unroll
    for (int nb = 0; nb < NB; nb++) {
        const int n = n0 + nb * 16 + li;
        const bool ok = n < g.N;
        const int j = ok ? n / g.nb : 0;
        brw[nb] = n - j * g.nb;
        const int64_t bo = ok ? boff[g.tab + j] : -1;
        bok[nb] = ok && brw[nb] < g.nvalid && bo >= 0;
        brow[nb] = B + (bok[nb] ? bo : 0);
        const int64_t co = ok ? coff[g.tab + j] : -1;
        cok[nb] = co >= 0;
        crow[nb] = C + (cok[nb] ? co + brw[nb] : 0);
    }
    struct Ops {
        f32x4 b[NB];
    };
    auto fetch = [&](Ops& o, int s) __attribute__((always_inline)) {
        const int kk = 16 * s + 4 * lh;
        const int sg = (kk >= g.seg[1]) + (kk >= g.seg[2]) + (kk >= g.seg[3]);
        const int p0 = sg == 0 ? 0 : sg == 1 ? g.seg[1] : sg == 2 ? g.seg[2] : g.seg[3];
        const int p1 = sg == 0 ? g.seg[1] : sg == 1 ? g.seg[2] : sg == 2 ? g.seg[3] : g.seg[4];
        const int64_t off = (int64_t)g.nb * p0 - p0;
#pragma unroll
        for (int nb = 0; nb < NB; nb++)
            if (nb < nbn)
                o.b[nb] = quad_or_zero<true>(brow[nb] + off + (int64_t)brw[nb] * (p1 - p0), kk, bok[nb] && kk < K, A);
    };
    f32x4 acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; mb++)
#pragma unroll
        for (int nb = 0; nb < NB; nb++) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    Ops o[PF + 1];
    if (nks > 0) {
        f32x4 v[2];
        stage_load(0, v);
        stage_store(0, v);
    }
#pragma unroll
    for (int s = 0; s < PF; s++)
        if (s < nks) fetch(o[s], s);
    __syncthreads();
    for (int s0 = 0; s0 < nks; s0 += PF + 1) {
#pragma unroll
        for (int r = 0; r <= PF; r++) {
            const int s = s0 + r;
            if (s < nks) {
                f32x4 vn[2];
                if (s + 1 < nks) stage_load(s + 1, vn);
                if (s + PF < nks) fetch(o[(r + PF) % (PF + 1)], s + PF);
                f32x4 af[MB];
#pragma unroll
                for (int mb = 0; mb < MB; mb++)
                    if (mb < nbm) af[mb] = as[s & 1][lh][mb * 16 + li];
#pragma unroll
                for (int q = 0; q < 4; q++)
#pragma unroll
                    for (int mb = 0; mb < MB; mb++)
#pragma unroll
                        for (int nb = 0; nb < NB; nb++)
                            if (mb < nbm && nb < nbn)
                                acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mb][q], o[r].b[nb][q],
                                                                                   acc[mb][nb], 0, 0, 0);
                if (s + 1 < nks) stage_store((s + 1) & 1, vn);
                __syncthreads();
            }
        }
    }
#pragma unroll
    for (int mb = 0; mb < MB; mb++)
#pragma unroll
        for (int nb = 0; nb < NB; nb++)
            if (mb < nbm && nb < nbn && cok[nb]) {
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int m = tl.m0 + mb * 16 + 4 * lh + v;
                    if (m < g.M) crow[nb][(int64_t)m * g.ldcm] = acc[mb][nb][v];
                }
            }
}

__global__ void reset_fused_counter(int* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

// Layout of the transposed U blocks: kept sector k occupies mp_k rows of
// ld[k] values (its site states' row ranges, each padded to a multiple of 4,
// start at pstart[k][s]), from off[k].
struct UtLayout {
    std::vector<int> ld;
    std::vector<std::vector<int>> pstart;  // -1 where the site state has no rows
    std::vector<int64_t> off;
    std::vector<UtSeg> segs;
    int64_t elems = 0;  // including the slack
    int max_ld = 0;
};

UtLayout ut_layout(const rot_blocked_problem* p, const Structure& st) {
    UtLayout L;
    L.ld.assign(p->n_new, 0);
    L.pstart.assign(p->n_new, std::vector<int>(p->d, -1));
    L.off.assign(p->n_new, 0);
    int64_t off = 0;
    for (int k = 0; k < p->n_new; k++) {
        const rot_sector& Q = p->new_sec[k];
        std::vector<std::pair<int, int>> rows;  // (s, rows of s)
        int ld = 0;
        for (int s = 0; s < p->d; s++) {
            if (st.rowstart[k][s] < 0) continue;
            const QN q{Q.n_up - p->site_qn[2 * s], Q.n_dn - p->site_qn[2 * s + 1]};
            const int len = p->old_sec[st.old_idx.at(q)].dim;
            L.pstart[k][s] = ld;
            rows.emplace_back(s, len);
            ld += (len + 3) / 4 * 4;
        }
        L.ld[k] = ld;
        L.max_ld = std::max(L.max_ld, ld);
        L.off[k] = off;
        for (auto [s, len] : rows) {
            UtSeg g{};
            g.u_off = p->U_off[k] + st.rowstart[k][s] * Q.dim;
            g.ut_off = off + L.pstart[k][s];
            g.rows = len;
            g.rows4 = (len + 3) / 4 * 4;
            g.mp = Q.dim;
            g.ld = ld;
            L.segs.push_back(g);
        }
        off += (int64_t)Q.dim * ld;
        const int64_t next = (off + 3) / 4 * 4;
        if (next > off) L.segs.push_back(UtSeg{0, off, 0, (int)(next - off), 1, 1});
        off = next;
    }
    L.elems = off + ut_slack(L.max_ld);
    L.segs.push_back(UtSeg{0, off, 0, (int)ut_slack(L.max_ld), 1, 1});
    return L;
}

// Workspace of the intermediate (elements): the stacked path's Xt (mQ rows
// of the padded row count of U^T_T per output block), which is never smaller
// than the grouped path's X (M_T x mQ per output block).
int64_t x_elements(const rot_blocked_problem* p, const Structure& st, const UtLayout& ut) {
    int64_t x = 0;
    for (int b = 0; b < p->n_ops; b++) {
        const int du = p->shift[2 * b], dd = p->shift[2 * b + 1];
        for (int k = 0; k < p->n_new; k++) {
            if (p->out_off[(int64_t)b * p->n_new + k] < 0) continue;
            const rot_sector& Q = p->new_sec[k];
            const int kt = st.new_idx.at(QN{Q.n_up + du, Q.n_dn + dd});
            x += ((int64_t)ut.ld[kt] * Q.dim + 63) / 64 * 64;
        }
    }
    return x;
}

struct FusedLists {
    std::vector<BlkTask> tasks;
    std::vector<BlkTerm> terms;
    int max_mT = 0;
    int max_k = 0;  // widest stage-1 K (old sector) of any term
};

void build_fused(const rot_blocked_problem* p, const Structure& st, const UtLayout& ut, FusedLists* F) {
    std::vector<std::pair<double, BlkTask>> work;
    std::vector<BlkTerm> terms;
    for (int b = 0; b < p->n_ops; b++) {
        const int du = p->shift[2 * b], dd = p->shift[2 * b + 1];
        for (int k = 0; k < p->n_new; k++) {
            const int64_t out_off = p->out_off[(int64_t)b * p->n_new + k];
            if (out_off < 0) continue;
            const rot_sector& Q = p->new_sec[k];
            const int kt = st.new_idx.at(QN{Q.n_up + du, Q.n_dn + dd});
            const rot_sector& Tsec = p->new_sec[kt];
            BlkTask task{};
            task.mT = Tsec.dim;
            task.mQ = Q.dim;
            task.term0 = (int)terms.size();
            task.ldT = ut.ld[kt];
            task.ldQ = ut.ld[k];
            task.uT_off = ut.off[kt];
            task.uQ_off = ut.off[k];
            task.out_off = out_off;
            double cost = 1.0;
            for (int s = 0; s < p->d; s++) {
                const int64_t rt = st.rowstart[kt][s], rq = st.rowstart[k][s];
                if (rt < 0 || rq < 0) continue;
                const QN qt{Tsec.n_up - p->site_qn[2 * s], Tsec.n_dn - p->site_qn[2 * s + 1]};
                const QN qs{qt.u - du, qt.d - dd};
                auto it = st.old_idx.find(qs);
                if (it == st.old_idx.end()) continue;
                const int64_t oo = p->O_off[(int64_t)b * p->n_old + it->second];
                if (oo < 0) continue;
                BlkTerm tm{};
                tm.a = p->old_sec[st.old_idx.at(qt)].dim;
                tm.k = p->old_sec[it->second].dim;
                tm.rt = ut.pstart[kt][s];
                tm.rq = ut.pstart[k][s];
                tm.o_off = oo;
                terms.push_back(tm);
                F->max_k = std::max(F->max_k, tm.k);
                cost += (double)tm.a * tm.k * Q.dim + (double)Tsec.dim * tm.a * Q.dim;
            }
            task.n_terms = (int)terms.size() - task.term0;
            F->max_mT = std::max(F->max_mT, task.mT);
            work.emplace_back(cost, task);
        }
    }
    // longest processing time first
    std::stable_sort(work.begin(), work.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    for (auto& w : work) F->tasks.push_back(w.second);
    F->terms = std::move(terms);
}

// Work-lists of the stacked path.  Xt offsets are relative to the workspace.
struct StackedLists {
    std::vector<StkGroup> g1, g2;      // streamed stage-1 groups (K > 80, or K = 0: zero rows); stage 2
    std::vector<StkTile> t1, t2, t2w;  // t2w: stage-2 workgroup tiles (128 columns)
    std::vector<StkGroupR> gr;         // stage 1 with resident operator rows
    std::vector<StkMember> mem;
    std::vector<StkTile> tr;
    std::vector<int64_t> boff, coff;
    std::vector<UtSeg> xzero;  // zero Xt segments (site states whose source sector is absent)
    int64_t x_elems = 0;
    bool ok = true;  // false: some kept sector has more than 4 site-state segments
};

void build_stacked(const rot_blocked_problem* p, const Structure& st, const UtLayout& ut, StackedLists* S) {
    std::vector<std::pair<int, int>> shifts;  // distinct shifts, first-appearance order
    for (int b = 0; b < p->n_ops; b++) {
        const std::pair<int, int> sh{p->shift[2 * b], p->shift[2 * b + 1]};
        if (std::find(shifts.begin(), shifts.end(), sh) == shifts.end()) shifts.push_back(sh);
    }
    // Xt block of (operator b, kept sector k): mQ rows of the padded row count
    // of U^T_T, allocated per (shift, kept sector) group, operators in order
    std::vector<int64_t> xbase((size_t)p->n_ops * p->n_new, -1);
    std::vector<std::pair<int, StkTile>> o1, o2, o2w, o_r;  // (work, tile): longest first
    for (int si = 0; si < (int)shifts.size(); si++) {
        const int du = shifts[si].first, dd = shifts[si].second;
        // Xt elements [gx0[k], gx1[k]) hold the blocks of kept sector k for this shift
        std::vector<int64_t> gx0(p->n_new, 0), gx1(p->n_new, 0);
        std::vector<int> ops;  // every operator of this shift
        for (int b = 0; b < p->n_ops; b++)
            if (p->shift[2 * b] == du && p->shift[2 * b + 1] == dd) ops.push_back(b);
        // stage 2 per kept sector Q (and the Xt blocks it reads)
        for (int k = 0; k < p->n_new; k++) {
            const rot_sector& Q = p->new_sec[k];
            auto itT = st.new_idx.find(QN{Q.n_up + du, Q.n_dn + dd});
            if (itT == st.new_idx.end()) continue;
            const int kt = itT->second;
            const rot_sector& T = p->new_sec[kt];
            std::vector<int> J;
            for (int b : ops)
                if (p->out_off[(int64_t)b * p->n_new + k] >= 0) J.push_back(b);
            if (J.empty()) continue;
            const int ldT = ut.ld[kt];
            const int n = (int)J.size();
            StkGroup g2{};
            g2.M = T.dim;
            g2.N = n * Q.dim;
            g2.K = ldT;
            g2.nb = g2.nvalid = Q.dim;
            g2.lda = ldT;
            g2.ldb = ldT;
            g2.ldcm = Q.dim;
            g2.a_off = ut.off[kt];
            g2.tab = (int64_t)S->boff.size();
            {
                int ns = 0;
                for (int s = 0; s < p->d; s++)
                    if (st.rowstart[kt][s] >= 0) {
                        if (ns == 4) {
                            S->ok = false;
                            break;
                        }
                        g2.seg[ns++] = ut.pstart[kt][s];
                    }
                g2.seg[ns] = ldT;
                for (int x = ns + 1; x < 5; x++) g2.seg[x] = kSegEnd;
            }
            gx0[k] = S->x_elems;
            for (int j = 0; j < n; j++) {
                const int64_t x = S->x_elems;
                S->x_elems += ((int64_t)Q.dim * ldT + 63) / 64 * 64;  // keep 256-byte alignment
                xbase[(size_t)J[j] * p->n_new + k] = x;
                S->boff.push_back(x);
                S->coff.push_back(p->out_off[(int64_t)J[j] * p->n_new + k]);
            }
            gx1[k] = S->x_elems;
            // the stage-1 stores address one group with 32-bit byte offsets
            if ((gx1[k] - gx0[k]) * (int64_t)sizeof(float) > kStkSpanMax) S->ok = false;
            const int gi2 = (int)S->g2.size();
            S->g2.push_back(g2);
            for (int m0 = 0; m0 < g2.M; m0 += 16 * kStkMB) {
                for (int n0 = 0; n0 < g2.N; n0 += 16 * kStkNB) o2.push_back({g2.K, StkTile{gi2, m0, n0, 0}});
                for (int n0 = 0; n0 < g2.N; n0 += kStk2Cols) o2w.push_back({g2.K, StkTile{gi2, m0, n0, 0}});
            }
            // Xt columns of site states whose source sector q_s = Q - qn(s) is
            // absent while q_s + Delta exists: zero, one run of m'_Q x a4 per
            // operator (the operators' Xt blocks are equally spaced)
            for (int s = 0; s < p->d; s++) {
                if (st.rowstart[kt][s] < 0 || st.rowstart[k][s] >= 0) continue;
                const QN qt{T.n_up - p->site_qn[2 * s], T.n_dn - p->site_qn[2 * s + 1]};
                const int a = p->old_sec[st.old_idx.at(qt)].dim;
                const int64_t spacing = ((int64_t)Q.dim * ldT + 63) / 64 * 64;
                S->xzero.push_back(UtSeg{0, xbase[(size_t)J[0] * p->n_new + k] + (int64_t)Q.dim * ut.pstart[kt][s], 0,
                                         Q.dim * ((a + 3) / 4 * 4), n, (int)spacing});
            }
        }
        // stage 1 per source sector q: every operator's block O(q + Delta <- q)
        // times U^T_Q of each site state s with Q = q + qn(s)
        for (int kq = 0; kq < p->n_old; kq++) {
            const rot_sector& q = p->old_sec[kq];
            auto itA = st.old_idx.find(QN{q.n_up + du, q.n_dn + dd});
            if (itA == st.old_idx.end()) continue;  // no operator block maps q anywhere kept
            const int a = p->old_sec[itA->second].dim, a4 = (a + 3) / 4 * 4;
            const int K = q.dim;
            const int n = (int)ops.size();
            struct Mem {
                int k, kt, s;
            };
            std::vector<Mem> ms;
            for (int s = 0; s < p->d; s++) {
                auto itQ = st.new_idx.find(QN{q.n_up + p->site_qn[2 * s], q.n_dn + p->site_qn[2 * s + 1]});
                if (itQ == st.new_idx.end()) continue;
                const int k = itQ->second;
                const rot_sector& Q = p->new_sec[k];
                auto itT = st.new_idx.find(QN{Q.n_up + du, Q.n_dn + dd});
                if (itT == st.new_idx.end()) continue;
                bool any = false;
                for (int b : ops) any = any || xbase[(size_t)b * p->n_new + k] >= 0;
                if (any) ms.push_back({k, itT->second, s});
            }
            if (ms.empty()) continue;
            const int64_t btab = (int64_t)S->boff.size();
            for (int b : ops) {
                S->boff.push_back(p->O_off[(int64_t)b * p->n_old + kq]);
                S->coff.push_back(-1);
            }
            // member tables: C offsets of (operator, Q) + first padded row of s
            auto member_tab = [&](const Mem& mm, int m0) {
                const int64_t tab = (int64_t)S->coff.size();
                for (int b : ops) {
                    const int64_t x = xbase[(size_t)b * p->n_new + mm.k];
                    S->boff.push_back(-1);
                    // Xt segment s of (b, Q): mQ x a4 row-major at mQ times the segment's first padded row
                    const int64_t seg0 = (int64_t)p->new_sec[mm.k].dim * ut.pstart[mm.kt][mm.s];
                    S->coff.push_back(x < 0 ? -1 : x + seg0 + (int64_t)m0 * a4);
                }
                return tab;
            };
            if (K <= 16 * kStkResK) {
                StkGroupR g{};
                g.N = n * a4;
                g.K = K;
                g.nb = a4;
                g.nvalid = a;
                g.tab = btab;
                const int mem0 = (int)S->mem.size();
                for (const Mem& mm : ms) {
                    const rot_sector& Q = p->new_sec[mm.k];
                    for (int m0 = 0; m0 < Q.dim; m0 += 16 * kStkMB) {
                        StkMember e{};
                        e.M = std::min(16 * kStkMB, Q.dim - m0);
                        e.lda = ut.ld[mm.k];
                        e.ldcm = a4;
                        e.a_off = ut.off[mm.k] + (int64_t)m0 * ut.ld[mm.k] + ut.pstart[mm.k][mm.s];
                        e.tab = member_tab(mm, m0);
                        e.c_base = gx0[mm.k];
                        e.span = (int)((gx1[mm.k] - gx0[mm.k]) * (int64_t)sizeof(float));
                        S->mem.push_back(e);
                    }
                }
                const int n_mem = (int)S->mem.size() - mem0;
                const int gi = (int)S->gr.size();
                S->gr.push_back(g);
                // workgroups of up to four members over 64 stacked columns
                for (int c0 = 0; c0 < n_mem; c0 += 4) {
                    const int cnt = std::min(4, n_mem - c0);
                    int work = 0;
                    for (int x = 0; x < cnt; x++) work = std::max(work, (S->mem[mem0 + c0 + x].M + 15) / 16);
                    work *= (K + 15) / 16;
                    for (int n0 = 0; n0 < g.N; n0 += 16 * kStkNB)
                        o_r.push_back({work, StkTile{gi, mem0 + c0, n0, cnt}});
                }
            } else {
                // wide source sectors: one streamed group per site state
                for (const Mem& mm : ms) {
                    const rot_sector& Q = p->new_sec[mm.k];
                    StkGroup g1{};
                    g1.M = Q.dim;
                    g1.N = n * a4;
                    g1.K = K;
                    g1.nb = a4;
                    g1.nvalid = a;
                    g1.lda = ut.ld[mm.k];
                    g1.ldb = K;
                    g1.ldcm = a4;
                    g1.a_off = ut.off[mm.k] + ut.pstart[mm.k][mm.s];
                    // B offsets: the operator blocks; C offsets: Xt blocks + first padded row of s
                    g1.tab = (int64_t)S->boff.size();
                    for (int b : ops) {
                        const int64_t x = xbase[(size_t)b * p->n_new + mm.k];
                        S->boff.push_back(p->O_off[(int64_t)b * p->n_old + kq]);
                        S->coff.push_back(x < 0 ? -1 : x + (int64_t)Q.dim * ut.pstart[mm.kt][mm.s]);
                    }
                    const int gi1 = (int)S->g1.size();
                    S->g1.push_back(g1);
                    for (int m0 = 0; m0 < g1.M; m0 += 16 * kStkMB)
                        for (int n0 = 0; n0 < g1.N; n0 += 16 * kStkNB) o1.push_back({K, StkTile{gi1, m0, n0, 0}});
                }
            }
        }
    }
    std::stable_sort(o1.begin(), o1.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    for (const auto& o : o1) S->t1.push_back(o.second);
    std::stable_sort(o2.begin(), o2.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    for (const auto& o : o2) S->t2.push_back(o.second);
    std::stable_sort(o2w.begin(), o2w.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    for (const auto& o : o2w) S->t2w.push_back(o.second);
    std::stable_sort(o_r.begin(), o_r.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    for (const auto& o : o_r) S->tr.push_back(o.second);
    // stage 1 reads the transposed-U area through one descriptor with 32-bit byte offsets
    if (ut.elems * (int64_t)sizeof(float) > kStkSpanMax) S->ok = false;
}

struct Lists {
    std::vector<GroupedProblem> p1, p2;
    int64_t x_elems = 0;
};

// Build the two problem lists; X offsets are relative to the workspace.
void build_lists(const rot_blocked_problem* p, const Structure& st, const float* ws, Lists* L) {
    for (int b = 0; b < p->n_ops; b++) {
        const int du = p->shift[2 * b], dd = p->shift[2 * b + 1];
        for (int k = 0; k < p->n_new; k++) {
            const int64_t out_off = p->out_off[(int64_t)b * p->n_new + k];
            if (out_off < 0) continue;
            const rot_sector& Q = p->new_sec[k];
            const int kt = st.new_idx.at(QN{Q.n_up + du, Q.n_dn + dd});
            const rot_sector& T = p->new_sec[kt];
            const int64_t x0 = L->x_elems;
            L->x_elems += (st.M[kt] * Q.dim + 63) / 64 * 64;  // keep 256-byte alignment
            for (int s = 0; s < p->d; s++) {
                const int64_t rt = st.rowstart[kt][s];
                if (rt < 0) continue;  // no rows of X for this s
                const QN qt{T.n_up - p->site_qn[2 * s], T.n_dn - p->site_qn[2 * s + 1]};
                const int kqt = st.old_idx.at(qt);
                GroupedProblem g{};
                g.M = p->old_sec[kqt].dim;
                g.N = Q.dim;
                g.c_off = x0 + rt * Q.dim;
                g.ldc = Q.dim;
                const QN qs{qt.u - du, qt.d - dd};
                auto it = st.old_idx.find(qs);
                const int64_t oo = it == st.old_idx.end() ? -1 : p->O_off[(int64_t)b * p->n_old + it->second];
                const int64_t rq = st.rowstart[k][s];
                if (oo >= 0 && rq >= 0) {
                    g.K = p->old_sec[it->second].dim;
                    g.a_off = oo;
                    g.lda = g.K;
                    g.b_off = p->U_off[k] + rq * Q.dim;
                    g.ldb = Q.dim;
                    const bool vec = aligned16(p->O_blk, g.a_off) && g.lda % 4 == 0 &&
                                     aligned16(p->U_blk, g.b_off) && g.ldb % 4 == 0;
                    g.flags = vec ? kGroupedVec : 0;
                } else {
                    g.K = 0;  // zero rows
                    g.lda = g.ldb = 1;
                }
                L->p1.push_back(g);
            }
            GroupedProblem g{};
            g.M = T.dim;
            g.N = Q.dim;
            g.K = (int)st.M[kt];
            g.a_off = p->U_off[kt];
            g.lda = T.dim;  // A(alpha, r) = U_T[r][alpha]
            g.b_off = x0;
            g.ldb = Q.dim;
            g.c_off = out_off;
            g.ldc = Q.dim;
            const bool vec = aligned16(p->U_blk, g.a_off) && g.lda % 4 == 0 && aligned16(ws, g.b_off) &&
                             g.ldb % 4 == 0;
            g.flags = vec ? kGroupedVec : 0;
            L->p2.push_back(g);
        }
    }
}

std::vector<GroupedTile> make_tiles(const std::vector<GroupedProblem>& probs, int edge) {
    std::vector<GroupedTile> t;
    for (int i = 0; i < (int)probs.size(); i++)
        for (int m0 = 0; m0 < probs[i].M; m0 += edge)
            for (int n0 = 0; n0 < probs[i].N; n0 += edge) t.push_back(GroupedTile{i, m0, n0, 0});
    // longest processing time first
    std::stable_sort(t.begin(), t.end(), [&](const GroupedTile& a, const GroupedTile& b) {
        return probs[a.prob].K > probs[b.prob].K;
    });
    return t;
}

struct DeviceLists {
    GroupedProblem* probs = nullptr;
    GroupedTile* tiles = nullptr;
    int n_tiles = 0;
};

struct Plan {
    DeviceLists s1, s2;
    int64_t counter_off = 0;  // bytes into the caller's workspace: the tile queue of this call
    int64_t x_elems = 0;
    BlkTask* f_tasks = nullptr;
    BlkTerm* f_terms = nullptr;
    UtSeg* f_segs = nullptr;
    int f_n_tasks = 0;
    int f_n_segs = 0;   // transpose segments (f_segs); the stacked path's zero Xt segments follow
    int k_n_xzero = 0;
    int f_max_mT = 0;
    int f_max_k = 0;
    int64_t ut_base = 0;   // transposed U area in the workspace (elements)
    int64_t ut_elems = 0;  // its size, slack included
    // stacked path: groups, tiles and per-operator tables of both stages
    StkGroup* k_g1 = nullptr;
    StkGroup* k_g2 = nullptr;
    StkTile* k_t1 = nullptr;
    StkTile* k_t2 = nullptr;
    int64_t* k_boff = nullptr;
    int64_t* k_coff = nullptr;
    StkGroupR* k_gr = nullptr;
    StkMember* k_mem = nullptr;
    StkTile* k_tr = nullptr;
    StkTile* k_t2w = nullptr;
    int k_n2w = 0;
    int k_n1 = 0, k_n2 = 0, k_nr = 0;
    bool k_ok = false;  // the stacked path applies
    // 0 grouped two-stage, 1 fused, 2 fused wide, 3/4 row-block operands
    // (narrow/wide), 5 stacked; -1 not chosen yet
    int path = -1;
    ~Plan() {
        (void)hipFree(k_g1);
        (void)hipFree(k_g2);
        (void)hipFree(k_t1);
        (void)hipFree(k_t2);
        (void)hipFree(k_boff);
        (void)hipFree(k_coff);
        (void)hipFree(k_gr);
        (void)hipFree(k_mem);
        (void)hipFree(k_tr);
        (void)hipFree(k_t2w);
        (void)hipFree(s1.probs);
        (void)hipFree(s1.tiles);
        (void)hipFree(s2.probs);
        (void)hipFree(s2.tiles);
        (void)hipFree(f_tasks);
        (void)hipFree(f_terms);
        (void)hipFree(f_segs);
    }
};

std::mutex g_mu;
PinnedLru<std::vector<unsigned char>, Plan> g_plans(kPlanCacheSize);

// Everything the work-lists depend on: the tables' contents, the shape, and
// the 16-byte alignment of the buffers (which decides vector loads).  The
// chosen path (fused or two grouped launches) is cached with the lists.  The
// pieces are handed to `f(bytes, size)` in a fixed order.
template <class F>
void walk_signature(const rot_blocked_problem* p, const void* ws, GroupedShape shape, F&& f) {
    auto put = [&](const auto* x, size_t n) { f(reinterpret_cast<const unsigned char*>(x), sizeof(*x) * n); };
    const int32_t head[4] = {p->d, p->n_old, p->n_new, p->n_ops};
    put(head, 4);
    const unsigned char align[4] = {
        (unsigned char)(reinterpret_cast<uintptr_t>(p->U_blk) & 15),
        (unsigned char)(reinterpret_cast<uintptr_t>(p->O_blk) & 15),
        (unsigned char)(reinterpret_cast<uintptr_t>(p->out_blk) & 15),
        (unsigned char)(reinterpret_cast<uintptr_t>(ws) & 15)};
    put(align, 4);
    put(&shape, 1);
    put(p->site_qn, 2 * (size_t)p->d);
    for (int k = 0; k < p->n_old; k++) {
        const int64_t v[4] = {p->old_sec[k].n_up, p->old_sec[k].n_dn, p->old_sec[k].dim, p->old_sec[k].offset};
        put(v, 4);
    }
    for (int k = 0; k < p->n_new; k++) {
        const int64_t v[4] = {p->new_sec[k].n_up, p->new_sec[k].n_dn, p->new_sec[k].dim, p->new_sec[k].offset};
        put(v, 4);
    }
    put(p->U_off, (size_t)p->n_new);
    if (p->n_ops > 0) {
        put(p->shift, 2 * (size_t)p->n_ops);
        put(p->O_off, (size_t)p->n_ops * p->n_old);
        put(p->out_off, (size_t)p->n_ops * p->n_new);
    }
}

std::vector<unsigned char> signature(const rot_blocked_problem* p, const void* ws, GroupedShape shape) {
    std::vector<unsigned char> v;
    walk_signature(p, ws, shape, [&](const unsigned char* b, size_t n) { v.insert(v.end(), b, b + n); });
    return v;
}

// Whether `key` is the signature of (p, ws, shape), compared piece by piece
// without building it.
bool signature_matches(const rot_blocked_problem* p, const void* ws, GroupedShape shape,
                       const std::vector<unsigned char>& key) {
    size_t at = 0;
    bool same = true;
    walk_signature(p, ws, shape, [&](const unsigned char* b, size_t n) {
        if (!same) return;
        same = at + n <= key.size() && (n == 0 || memcmp(key.data() + at, b, n) == 0);
        at += n;
    });
    return same && at == key.size();
}

hipError_t upload(const std::vector<GroupedProblem>& probs, const std::vector<GroupedTile>& tiles, DeviceLists* d) {
    d->n_tiles = (int)tiles.size();
    if (probs.empty() || tiles.empty()) return hipSuccess;
    hipError_t e = hipMalloc(&d->probs, sizeof(GroupedProblem) * probs.size());
    if (e == hipSuccess) e = hipMalloc(&d->tiles, sizeof(GroupedTile) * tiles.size());
    if (e == hipSuccess)
        e = hipMemcpy(d->probs, probs.data(), sizeof(GroupedProblem) * probs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(d->tiles, tiles.data(), sizeof(GroupedTile) * tiles.size(), hipMemcpyHostToDevice);
    return e;
}

GroupedShape blocked_shape() { return GroupedShape::k32; }

// Bytes of X (grouped path) and the transposed U blocks (fused path); the
// call's tile-queue counter follows, 256-byte aligned.
int64_t counter_offset(int64_t x_elems, int64_t ut_elems) {
    return ((x_elems + 63) / 64 * 64 + ut_elems) * (int64_t)sizeof(float) / 256 * 256 + 256;
}

}  // namespace

// X of the grouped path, then the transposed U blocks of the fused path, then
// the call's tile-queue counter (in the caller's workspace, so calls with
// different workspaces never share a queue).
size_t blocked_workspace_bytes(const rot_blocked_problem* p) {
    Structure st;
    std::string why;
    if (!build_structure(p, &st, &why)) return 0;
    const UtLayout ut = ut_layout(p, st);
    return (size_t)counter_offset(x_elements(p, st, ut), ut.elems) + 256;
}

rot_status blocked_validate(const rot_blocked_problem* p, std::string* why) {
    Structure st;
    return build_structure(p, &st, why) ? ROT_OK : ROT_ERR_INVALID_ARG;
}

namespace {

hipError_t run_grouped(const rot_blocked_problem* p, Plan* plan, void* ws, GroupedShape shape, hipStream_t stream) {
    GroupedLaunch a{};
    a.a_base = p->O_blk;
    a.b_base = p->U_blk;
    a.c_base = static_cast<float*>(ws);
    a.probs = plan->s1.probs;
    a.tiles = plan->s1.tiles;
    a.n_tiles = plan->s1.n_tiles;
    a.a_kcontig = true;   // O block (rows x cols), K = its columns
    a.b_kcontig = false;  // U_Q rows: B(k, n) = U_Q[row k][n]
    a.dynamic = true;
    a.shape = shape;
    a.grid = 2048;  // persistent: 8 single-wave workgroups per CU
    a.counter = reinterpret_cast<int*>(static_cast<char*>(ws) + plan->counter_off);
    hipError_t e = prof_timed("blocked_stage1_fp32", stream, [&] { return grouped_gemm_f32(a, stream); });
    if (e != hipSuccess) return e;
    GroupedLaunch b = a;
    b.a_base = p->U_blk;
    b.b_base = static_cast<const float*>(ws);
    b.c_base = p->out_blk;
    b.probs = plan->s2.probs;
    b.tiles = plan->s2.tiles;
    b.n_tiles = plan->s2.n_tiles;
    b.a_kcontig = false;  // A(alpha, r) = U_T[r][alpha]
    b.b_kcontig = false;  // X[r][beta]
    return prof_timed("blocked_stage2_fp32", stream, [&] { return grouped_gemm_f32(b, stream); });
}

// Fused variants: (register set of output row blocks, column blocks per
// pass); `wide` keeps every column block of a task in one pass (fewest
// operand fetches), otherwise fewer per pass (more resident waves).
template <int MAXA, int CG>
void launch_fused(Plan* plan, const float* ut, const rot_blocked_problem* p, int* counter, hipStream_t stream) {
    const int grid = 256 * 4;  // 4 workgroups of 4 waves per CU, each wave a task queue consumer
    hipLaunchKernelGGL((blocked_fused_kernel<MAXA, CG>), dim3(grid), dim3(256), 0, stream, plan->f_tasks,
                       plan->f_n_tasks, plan->f_terms, ut, p->O_blk, p->out_blk, counter);
}

template <int MAXA, int CG>
void launch_rowblock(Plan* plan, const float* ut, const rot_blocked_problem* p, int* counter, hipStream_t stream) {
    const int grid = 256 * 4;
    hipLaunchKernelGGL((blocked_rowblock_kernel<MAXA, CG, MAXA>), dim3(grid), dim3(256), 0, stream, plan->f_tasks,
                       plan->f_n_tasks, plan->f_terms, ut, p->O_blk, p->out_blk, counter);
}

// The row-block variant holds up to 16 * MAXA stage-1 K values per lane
// (MAXA = 4 or 5: output and stage-1 extents up to 64 or 80).
bool rowblock_ok(const Plan* plan) {
    return plan->f_max_mT <= 80 && plan->f_max_k <= (plan->f_max_mT <= 64 ? 64 : 80);
}

hipError_t run_fused(const rot_blocked_problem* p, Plan* plan, bool wide, bool rowblock, void* ws,
                     hipStream_t stream) {
    if (plan->f_n_tasks == 0) return hipSuccess;
    hipError_t e = prof_timed("blocked_transpose_u", stream, [&] {
        hipLaunchKernelGGL(transpose_u_kernel, dim3(16, (unsigned)plan->f_n_segs), dim3(256), 0, stream,
                           plan->f_segs, p->U_blk, static_cast<float*>(ws));
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    float* ut = static_cast<float*>(ws) + plan->ut_base;
    int* counter = reinterpret_cast<int*>(static_cast<char*>(ws) + plan->counter_off);
    return prof_timed("blocked_fused_fp32", stream, [&] {
        hipLaunchKernelGGL(reset_fused_counter, dim3(1), dim3(64), 0, stream, counter);
        if (rowblock) {
            if (plan->f_max_mT <= 64) {
                if (wide) launch_rowblock<4, 4>(plan, ut, p, counter, stream); else launch_rowblock<4, 2>(plan, ut, p, counter, stream);
            } else {
                if (wide) launch_rowblock<5, 3>(plan, ut, p, counter, stream); else launch_rowblock<5, 2>(plan, ut, p, counter, stream);
            }
        } else if (plan->f_max_mT <= 64) {
            if (wide) launch_fused<4, 4>(plan, ut, p, counter, stream); else launch_fused<4, 2>(plan, ut, p, counter, stream);
        } else if (plan->f_max_mT <= 80) {
            if (wide) launch_fused<5, 3>(plan, ut, p, counter, stream); else launch_fused<5, 2>(plan, ut, p, counter, stream);
        } else {
            if (wide) launch_fused<8, 3>(plan, ut, p, counter, stream); else launch_fused<8, 2>(plan, ut, p, counter, stream);
        }
        return hipGetLastError();
    });
}

// The streamed kernel's launch: 32 columns per wave, two k steps in flight.
template <bool BVEC>
hipError_t launch_stacked(const StkTile* tiles, int n, const StkGroup* groups, const Plan* plan, const float* A,
                          const float* B, float* C, hipStream_t stream) {
    constexpr int NB = 2, PF = 2;
    // stage 2 (aligned B) reads the segment-ordered Xt blocks
    const int waves = n * (kStkNB / NB);
    hipLaunchKernelGGL((blocked_stacked_kernel<NB, PF, BVEC, BVEC>), dim3((waves + 3) / 4), dim3(256), 0, stream,
                       tiles, n, groups, plan->k_boff, plan->k_coff, A, B, C);
    return hipGetLastError();
}

// ROT_STK2=wave: stage 2 on the streamed kernel (one wave per tile, U^T_T
// from L2) instead of the workgroup kernel; a measurement switch.
bool stage2_per_wave() {
    const char* e = getenv("ROT_STK2");
    return e && strcmp(e, "wave") == 0;
}

// Transposed U blocks into the workspace together with the zero Xt segments,
// then the two stacked launches (stage 1 writes every other element of Xt
// that stage 2 reads, padding included).
hipError_t run_stacked(const rot_blocked_problem* p, Plan* plan, void* ws, hipStream_t stream) {
    if (plan->k_n2 == 0) return hipSuccess;
    float* ut = static_cast<float*>(ws) + plan->ut_base;
    float* xt = static_cast<float*>(ws);
    hipError_t e = prof_timed("blocked_transpose_u", stream, [&] {
        hipLaunchKernelGGL(transpose_u_kernel, dim3(16, (unsigned)(plan->f_n_segs + plan->k_n_xzero)), dim3(256),
                           0, stream, plan->f_segs, p->U_blk, xt);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    e = prof_timed("blocked_stacked1_fp32", stream, [&] {
        if (plan->k_nr > 0)
            hipLaunchKernelGGL(blocked_stacked_lds_kernel<1>, dim3(plan->k_nr), dim3(512), 0, stream, plan->k_tr,
                               plan->k_gr, plan->k_mem, plan->k_boff, plan->k_coff, ut, p->O_blk, xt,
                               (int)(plan->ut_elems * (int64_t)sizeof(float)));
        if (plan->k_n1 > 0)
            return launch_stacked<false>(plan->k_t1, plan->k_n1, plan->k_g1, plan, ut, p->O_blk, xt, stream);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    return prof_timed("blocked_stacked2_fp32", stream, [&] {
        if (stage2_per_wave())
            return launch_stacked<true>(plan->k_t2, plan->k_n2, plan->k_g2, plan, ut, xt, p->out_blk, stream);
        hipLaunchKernelGGL(blocked_stacked2_wg_kernel, dim3(plan->k_n2w), dim3(256), 0, stream, plan->k_t2w,
                           plan->k_g2, plan->k_boff, plan->k_coff, ut, xt, p->out_blk,
                           (int)(plan->ut_elems * (int64_t)sizeof(float)));
        return hipGetLastError();
    });
}

// Paths: 0 two grouped launches, 1 fused (narrow passes), 2 fused (wide),
// 3 / 4 the fused kernel with whole row blocks of operator rows (narrow /
// wide), 5 two stacked launches.  ROT_BLOCKED_PATH = grouped | fused |
// fused_wide | rowblock | rowblock_wide | stacked forces one; otherwise every
// applicable path is timed once per block structure and the fastest is kept.
int forced_path() {
    const char* e = getenv("ROT_BLOCKED_PATH");
    if (!e) return -1;
    if (!strcmp(e, "grouped")) return 0;
    if (!strcmp(e, "fused")) return 1;
    if (!strcmp(e, "fused_wide")) return 2;
    if (!strcmp(e, "rowblock")) return 3;
    if (!strcmp(e, "rowblock_wide")) return 4;
    if (!strcmp(e, "stacked")) return 5;
    return -1;
}

hipError_t run_path(const rot_blocked_problem* p, Plan* plan, void* ws, GroupedShape shape, int path,
                    hipStream_t stream) {
    if (path == 0) return run_grouped(p, plan, ws, shape, stream);
    if (path == 5) return run_stacked(p, plan, ws, stream);
    return run_fused(p, plan, path == 2 || path == 4, path >= 3, ws, stream);
}

}  // namespace

hipError_t rotate_blocked(const rot_blocked_problem* p, void* ws, size_t ws_bytes, hipStream_t stream) {
    (void)ws_bytes;
    if (p->n_ops == 0) return hipSuccess;
    const GroupedShape shape = blocked_shape();
    const int forced = forced_path();
    // Under stream capture the graph keeps the plan's device work-lists: the
    // plan is pinned (never evicted), and a structure not seen before cannot
    // be planned (its lists are copied to the device synchronously).
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    const bool capturing = hipStreamIsCapturing(stream, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone;
    std::lock_guard<std::mutex> lk(g_mu);
    Plan* plan = g_plans.find_if(
        [&](const std::vector<unsigned char>& key) { return signature_matches(p, ws, shape, key); });
    if (!plan && capturing) {
        set_error(ROT_ERR_UNSUPPORTED,
                  "rot_batch_blocked: the first call for a block structure must run outside stream capture "
                  "(it builds and uploads the work-lists); call it once eagerly before capturing");
        return hipErrorStreamCaptureUnsupported;
    }
    if (!plan) {
        Structure st;
        std::string why;
        if (!build_structure(p, &st, &why)) return hipErrorInvalidValue;  // validated by the caller
        Lists L;
        build_lists(p, st, static_cast<const float*>(ws), &L);
        const UtLayout ut = ut_layout(p, st);
        FusedLists F;
        build_fused(p, st, ut, &F);
        StackedLists S;
        build_stacked(p, st, ut, &S);
        auto np = std::make_unique<Plan>();
        np->x_elems = std::max(L.x_elems, S.x_elems);
        const int edge = grouped_tile_edge(shape);
        hipError_t e = upload(L.p1, make_tiles(L.p1, edge), &np->s1);
        if (e == hipSuccess) e = upload(L.p2, make_tiles(L.p2, edge), &np->s2);
        np->f_n_tasks = (int)F.tasks.size();
        np->f_max_mT = F.max_mT;
        np->f_max_k = F.max_k;
        np->f_n_segs = (int)ut.segs.size();
        np->ut_base = (np->x_elems + 63) / 64 * 64;
        np->ut_elems = ut.elems;
        np->counter_off = counter_offset(np->x_elems, ut.elems);
        // the transpose segments (offsets from the workspace base), then the
        // stacked path's zero Xt segments
        std::vector<UtSeg> segs = ut.segs;
        for (UtSeg& g : segs) g.ut_off += np->ut_base;
        if (S.ok) segs.insert(segs.end(), S.xzero.begin(), S.xzero.end());
        np->k_n_xzero = S.ok ? (int)S.xzero.size() : 0;
        if (e == hipSuccess && !segs.empty()) e = hipMalloc(&np->f_segs, sizeof(UtSeg) * segs.size());
        if (e == hipSuccess && !segs.empty())
            e = hipMemcpy(np->f_segs, segs.data(), sizeof(UtSeg) * segs.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess && !F.tasks.empty()) e = hipMalloc(&np->f_tasks, sizeof(BlkTask) * F.tasks.size());
        if (e == hipSuccess && !F.terms.empty()) e = hipMalloc(&np->f_terms, sizeof(BlkTerm) * F.terms.size());
        if (e == hipSuccess && !F.tasks.empty())
            e = hipMemcpy(np->f_tasks, F.tasks.data(), sizeof(BlkTask) * F.tasks.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess && !F.terms.empty())
            e = hipMemcpy(np->f_terms, F.terms.data(), sizeof(BlkTerm) * F.terms.size(), hipMemcpyHostToDevice);
        np->k_n1 = (int)S.t1.size();
        np->k_n2 = (int)S.t2.size();
        np->k_nr = (int)S.tr.size();
        np->k_n2w = (int)S.t2w.size();
        np->k_ok = S.ok;
        auto up = [&](auto** dst, const auto& v) {
            if (e != hipSuccess || v.empty()) return;
            e = hipMalloc(dst, sizeof(v[0]) * v.size());
            if (e == hipSuccess) e = hipMemcpy(*dst, v.data(), sizeof(v[0]) * v.size(), hipMemcpyHostToDevice);
        };
        up(&np->k_g1, S.g1);
        up(&np->k_g2, S.g2);
        up(&np->k_t1, S.t1);
        up(&np->k_t2, S.t2);
        up(&np->k_boff, S.boff);
        up(&np->k_coff, S.coff);
        up(&np->k_gr, S.gr);
        up(&np->k_mem, S.mem);
        up(&np->k_tr, S.tr);
        up(&np->k_t2w, S.t2w);
        if (e != hipSuccess) return e;
        plan = g_plans.insert(signature(p, ws, shape), std::move(np));
    }
    // paths that apply to this structure: the fused kernels keep at most
    // 8 x 16 output rows per lane set
    std::vector<int> paths{0};
    if (plan->f_max_mT <= 128) {
        paths.push_back(1);
        paths.push_back(2);
        if (rowblock_ok(plan)) {
            paths.push_back(3);
            paths.push_back(4);
        }
    }
    if (plan->k_ok) paths.push_back(5);
    if (capturing) {
        g_plans.pin(plan);
        // no timing under capture: the stacked path, or the grouped one
        if (plan->path < 0 && forced < 0) plan->path = plan->k_ok ? 5 : 0;
    }
    int path = forced >= 0 ? forced : plan->path;
    if (path >= 0 && std::find(paths.begin(), paths.end(), path) == paths.end()) {
        // a forced path that does not apply: the closest one that does
        if ((path == 3 || path == 4) && plan->f_max_mT <= 128) path -= 2;
        else path = plan->k_ok ? 5 : 0;
    }
    if (path < 0) {
        // time each applicable path (second run, after a warm-up run)
        const int n_paths = (int)paths.size();
        std::vector<hipEvent_t> ev(n_paths + 1, nullptr);
        hipError_t e = hipSuccess;
        for (int i = 0; i <= n_paths && e == hipSuccess; i++) e = hipEventCreate(&ev[i]);
        for (int rep = 0; rep < 2 && e == hipSuccess; rep++) {
            for (int q = 0; q < n_paths && e == hipSuccess; q++) {
                e = hipEventRecord(ev[q], stream);
                if (e == hipSuccess) e = run_path(p, plan, ws, shape, paths[q], stream);
            }
            if (e == hipSuccess) e = hipEventRecord(ev[n_paths], stream);
        }
        float best = 1e30f;
        int best_q = 0;
        if (e == hipSuccess) e = hipEventSynchronize(ev[n_paths]);
        for (int q = 0; q < n_paths && e == hipSuccess; q++) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[q], ev[q + 1]);
            log_msg(3, "blocked structure of %d operators: path %d %.3f ms", p->n_ops, paths[q], ms);
            if (ms < best) {
                best = ms;
                best_q = q;
            }
        }
        for (hipEvent_t x : ev)
            if (x) (void)hipEventDestroy(x);
        if (e != hipSuccess) return e;
        plan->path = paths[best_q];
        log_msg(2, "blocked structure of %d operators: execution path %d (%.3f ms when timed)", p->n_ops,
                plan->path, best);
        // the chosen path writes the result, so this call matches every later
        // one bit for bit (the paths sum in different orders)
        path = plan->path;
    }
    return run_path(p, plan, ws, shape, path, stream);
}

}  // namespace rot
