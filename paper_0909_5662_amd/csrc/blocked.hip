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
#include <vector>

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
// One site state's rows of one kept sector in the transposed-U area.
struct UtSeg {
    int64_t u_off;   // first row of the segment in U_blk (leading dimension mp)
    int64_t ut_off;  // U^T area offset of column 0 of this segment (leading dimension ld)
    int rows, rows4, mp, ld;
};

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));

// Slack after the transposed-U area: stage 1 reads up to CG - 1 column
// blocks (and a partial one) past a sector, i.e. fewer than 96 rows of the
// widest block, and padded k runs past a row by fewer than 16 values.  The
// whole area, slack and alignment gaps included, is zero before the
// transpose fills it, so such reads only ever meet finite values.
inline int64_t ut_slack(int max_ld) { return 96 * (int64_t)max_ld + 64; }

__global__ __launch_bounds__(256) void transpose_u_kernel(const UtSeg* __restrict__ segs, const float* __restrict__ U,
                                                          float* __restrict__ Ut) {
    const UtSeg g = segs[blockIdx.y];
    const int64_t n = (int64_t)g.rows4 * g.mp;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int i = (int)(e / g.mp), beta = (int)(e % g.mp);
        Ut[g.ut_off + (int64_t)beta * g.ld + i] = i < g.rows ? U[g.u_off + (int64_t)i * g.mp + beta] : 0.f;
    }
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
                        f32x4 av;
                        if (rok && kk + 4 <= tm.k) {
                            av = *reinterpret_cast<const f32x4u*>(orow + kk);
                        } else {
#pragma unroll
                            for (int j = 0; j < 4; j++) av[j] = (rok && kk + j < tm.k) ? orow[kk + j] : 0.f;
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
// (term, row block) pair at once, before the pair's first U^T_Q values: the
// operator block comes from HBM, and with every k step's rows requested
// together the pair waits for one HBM round trip instead of one per 16-wide
// k step.  U^T_Q values (L2-resident) are still fetched one k step ahead.
// Needs every term's stage-1 K <= 16 * KS.
template <int MAXA, int CG, int KS>
__global__ __launch_bounds__(256) void blocked_rowblock_kernel(const BlkTask* __restrict__ tasks, int n_tasks,
                                                               const BlkTerm* __restrict__ terms,
                                                               const float* __restrict__ Ut,
                                                               const float* __restrict__ O, float* __restrict__ out,
                                                               int* __restrict__ counter) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lh = lane >> 4;
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
            for (int e = 0; e < T.n_terms; e++) {
                const BlkTerm tm = terms[T.term0 + e];
                const int nks = (tm.k + 15) >> 4;
                for (int rb = 0; rb * 16 < tm.a; rb++) {
                    f32x4 ut[MAXA];
#pragma unroll
                    for (int ca = 0; ca < MAXA; ca++)
                        if (ca < nba)
                            ut[ca] = *reinterpret_cast<const f32x4*>(uT + (int64_t)(ca * 16 + li) * T.ldT + tm.rt +
                                                                     rb * 16 + 4 * lh);
                    // the row block's operator rows, every k step
                    const int row = rb * 16 + li;
                    const bool rok = row < tm.a;
                    const float* orow = O + tm.o_off + (int64_t)row * tm.k;
                    f32x4 a[KS];
#pragma unroll
                    for (int ks = 0; ks < KS; ks++) {
                        const int kk = ks * 16 + 4 * lh;
                        if (ks < nks) {
                            if (rok && kk + 4 <= tm.k) {
                                a[ks] = *reinterpret_cast<const f32x4u*>(orow + kk);
                            } else {
#pragma unroll
                                for (int j = 0; j < 4; j++) a[ks][j] = (rok && kk + j < tm.k) ? orow[kk + j] : 0.f;
                            }
                        }
                    }
                    f32x4 x[CG], bv[CG];
#pragma unroll
                    for (int c = 0; c < CG; c++) x[c] = f32x4{0.f, 0.f, 0.f, 0.f};
                    if (nks > 0) {
#pragma unroll
                        for (int c = 0; c < CG; c++)
                            bv[c] = *reinterpret_cast<const f32x4*>(uQ + (int64_t)((cg0 + c) * 16 + li) * T.ldQ +
                                                                    tm.rq + 4 * lh);
                    }
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
                }
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
        off = (off + 3) / 4 * 4;
    }
    L.elems = off + ut_slack(L.max_ld);
    return L;
}

// Workspace of the grouped path's intermediate X (elements).
int64_t x_elements(const rot_blocked_problem* p, const Structure& st) {
    int64_t x = 0;
    for (int b = 0; b < p->n_ops; b++) {
        const int du = p->shift[2 * b], dd = p->shift[2 * b + 1];
        for (int k = 0; k < p->n_new; k++) {
            if (p->out_off[(int64_t)b * p->n_new + k] < 0) continue;
            const rot_sector& Q = p->new_sec[k];
            const int kt = st.new_idx.at(QN{Q.n_up + du, Q.n_dn + dd});
            x += (st.M[kt] * Q.dim + 63) / 64 * 64;
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
    int f_n_segs = 0;
    int f_max_mT = 0;
    int f_max_k = 0;
    int64_t ut_base = 0;   // transposed U area in the workspace (elements)
    int64_t ut_elems = 0;  // its size, slack included
    int path = -1;  // 0 grouped two-stage, 1 fused, 2 fused wide, 3/4 row-block operands (narrow/wide); -1 not chosen yet
    ~Plan() {
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

template <class T>
void put(std::vector<unsigned char>& v, const T* p, size_t n) {
    const unsigned char* c = reinterpret_cast<const unsigned char*>(p);
    v.insert(v.end(), c, c + sizeof(T) * n);
}

// Everything the work-lists depend on: the tables' contents, the shape, and
// the 16-byte alignment of the buffers (which decides vector loads).  The
// chosen path (fused or two grouped launches) is cached with the lists.
std::vector<unsigned char> signature(const rot_blocked_problem* p, const void* ws, GroupedShape shape) {
    std::vector<unsigned char> v;
    const int32_t head[4] = {p->d, p->n_old, p->n_new, p->n_ops};
    put(v, head, 4);
    const unsigned char align[4] = {
        (unsigned char)(reinterpret_cast<uintptr_t>(p->U_blk) & 15),
        (unsigned char)(reinterpret_cast<uintptr_t>(p->O_blk) & 15),
        (unsigned char)(reinterpret_cast<uintptr_t>(p->out_blk) & 15),
        (unsigned char)(reinterpret_cast<uintptr_t>(ws) & 15)};
    put(v, align, 4);
    put(v, &shape, 1);
    put(v, p->site_qn, 2 * p->d);
    for (int k = 0; k < p->n_old; k++) {
        const int64_t f[4] = {p->old_sec[k].n_up, p->old_sec[k].n_dn, p->old_sec[k].dim, p->old_sec[k].offset};
        put(v, f, 4);
    }
    for (int k = 0; k < p->n_new; k++) {
        const int64_t f[4] = {p->new_sec[k].n_up, p->new_sec[k].n_dn, p->new_sec[k].dim, p->new_sec[k].offset};
        put(v, f, 4);
    }
    put(v, p->U_off, p->n_new);
    if (p->n_ops > 0) {
        put(v, p->shift, 2 * (size_t)p->n_ops);
        put(v, p->O_off, (size_t)p->n_ops * p->n_old);
        put(v, p->out_off, (size_t)p->n_ops * p->n_new);
    }
    return v;
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
    return (size_t)counter_offset(x_elements(p, st), ut_layout(p, st).elems) + 256;
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
    float* ut = static_cast<float*>(ws) + plan->ut_base;
    hipError_t e = prof_timed("blocked_transpose_u", stream, [&] {
        hipError_t err = fill_zero(ut, plan->ut_elems * (int64_t)sizeof(float), stream);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(transpose_u_kernel, dim3(16, (unsigned)plan->f_n_segs), dim3(256), 0, stream,
                           plan->f_segs, p->U_blk, ut);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
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

// Paths: 0 two grouped launches, 1 fused (narrow passes), 2 fused (wide),
// 3 / 4 the fused kernel with whole row blocks of operator rows (narrow /
// wide).  ROT_BLOCKED_PATH = grouped | fused | fused_wide | rowblock |
// rowblock_wide forces one; otherwise every applicable path is timed once
// per block structure and the fastest is kept.
int forced_path() {
    const char* e = getenv("ROT_BLOCKED_PATH");
    if (!e) return -1;
    if (!strcmp(e, "grouped")) return 0;
    if (!strcmp(e, "fused")) return 1;
    if (!strcmp(e, "fused_wide")) return 2;
    if (!strcmp(e, "rowblock")) return 3;
    if (!strcmp(e, "rowblock_wide")) return 4;
    return -1;
}

hipError_t run_path(const rot_blocked_problem* p, Plan* plan, void* ws, GroupedShape shape, int path,
                    hipStream_t stream) {
    if (path == 0) return run_grouped(p, plan, ws, shape, stream);
    return run_fused(p, plan, path == 2 || path == 4, path >= 3, ws, stream);
}

}  // namespace

hipError_t rotate_blocked(const rot_blocked_problem* p, void* ws, size_t ws_bytes, hipStream_t stream) {
    (void)ws_bytes;
    if (p->n_ops == 0) return hipSuccess;
    const GroupedShape shape = blocked_shape();
    const int forced = forced_path();
    std::vector<unsigned char> sig = signature(p, ws, shape);
    // Under stream capture the graph keeps the plan's device work-lists: the
    // plan is pinned (never evicted), and a structure not seen before cannot
    // be planned (its lists are copied to the device synchronously).
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    const bool capturing = hipStreamIsCapturing(stream, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone;
    std::lock_guard<std::mutex> lk(g_mu);
    Plan* plan = g_plans.find(sig);
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
        auto np = std::make_unique<Plan>();
        np->x_elems = L.x_elems;
        const int edge = grouped_tile_edge(shape);
        hipError_t e = upload(L.p1, make_tiles(L.p1, edge), &np->s1);
        if (e == hipSuccess) e = upload(L.p2, make_tiles(L.p2, edge), &np->s2);
        np->f_n_tasks = (int)F.tasks.size();
        np->f_max_mT = F.max_mT;
        np->f_max_k = F.max_k;
        np->f_n_segs = (int)ut.segs.size();
        np->ut_base = (L.x_elems + 63) / 64 * 64;
        np->ut_elems = ut.elems;
        np->counter_off = counter_offset(L.x_elems, ut.elems);
        if (e == hipSuccess && !ut.segs.empty()) e = hipMalloc(&np->f_segs, sizeof(UtSeg) * ut.segs.size());
        if (e == hipSuccess && !ut.segs.empty())
            e = hipMemcpy(np->f_segs, ut.segs.data(), sizeof(UtSeg) * ut.segs.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess && !F.tasks.empty()) e = hipMalloc(&np->f_tasks, sizeof(BlkTask) * F.tasks.size());
        if (e == hipSuccess && !F.terms.empty()) e = hipMalloc(&np->f_terms, sizeof(BlkTerm) * F.terms.size());
        if (e == hipSuccess && !F.tasks.empty())
            e = hipMemcpy(np->f_tasks, F.tasks.data(), sizeof(BlkTask) * F.tasks.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess && !F.terms.empty())
            e = hipMemcpy(np->f_terms, F.terms.data(), sizeof(BlkTerm) * F.terms.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return e;
        if (F.max_mT > 128) np->path = 0;  // the fused kernel keeps at most 8 x 16 output rows per lane set
        plan = g_plans.insert(std::move(sig), std::move(np));
    }
    if (capturing) {
        g_plans.pin(plan);
        // no timing under capture: the fused path unless the structure needs the grouped one
        if (plan->path < 0 && forced < 0) plan->path = plan->f_max_mT > 128 ? 0 : 1;
    }
    int path = forced >= 0 ? forced : plan->path;
    if (path >= 3 && !rowblock_ok(plan)) path = path - 2;
    if (path >= 1 && plan->f_max_mT > 128) path = 0;
    if (path < 0) {
        // time each applicable path (second run, after a warm-up run)
        const int n_paths = plan->f_max_mT > 128 ? 1 : rowblock_ok(plan) ? 5 : 3;
        hipEvent_t ev[6];
        hipError_t e = hipSuccess;
        for (int i = 0; i < 6 && e == hipSuccess; i++) e = hipEventCreate(&ev[i]);
        for (int rep = 0; rep < 2 && e == hipSuccess; rep++) {
            for (int q = 0; q < n_paths && e == hipSuccess; q++) {
                e = hipEventRecord(ev[q], stream);
                if (e == hipSuccess) e = run_path(p, plan, ws, shape, q, stream);
            }
            if (e == hipSuccess) e = hipEventRecord(ev[n_paths], stream);
        }
        float best = 1e30f;
        int best_q = 0;
        if (e == hipSuccess) e = hipEventSynchronize(ev[n_paths]);
        for (int q = 0; q < n_paths && e == hipSuccess; q++) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[q], ev[q + 1]);
            if (ms < best) {
                best = ms;
                best_q = q;
            }
        }
        for (int i = 0; i < 6; i++) (void)hipEventDestroy(ev[i]);
        if (e != hipSuccess) return e;
        plan->path = best_q;
        log_msg(2, "blocked structure of %d operators: execution path %d (%.3f ms when timed)", p->n_ops, best_q,
                best);
        // the chosen path writes the result, so this call matches every later
        // one bit for bit (the paths sum in different orders)
        path = best_q;
    }
    return run_path(p, plan, ws, shape, path, stream);
}

}  // namespace rot
