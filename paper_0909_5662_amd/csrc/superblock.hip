// The superblock Hamiltonian applied to a state over quantum-number blocks
// (Eq. (9) and Eq. (10)): out = sum_l coef_l (O_B (x) O_a (x) O_a~ (x) O_B~) psi.
//
// The state is one dense block per system sector Q of [B a] (rows: site a
// state s slow, B state fast) paired with environment sector P = target - Q of
// [a~ B~] (columns: site a~ state t slow, B~ state fast).  Inside a block the
// rows split into segments (s, q) of B sector q = Q - qn(s) and the columns into
// segments (t, p).  A term maps source segment (s, q) x (t, p) to output
// segment (s', q + dB) x (t', p + dB~) with weight site_a[s'][s] site_at[t'][t]:
//   operator on B:  out_seg += w coef O_B(q' <- q) psi_seg        (K = dim q)
//   operator on B~: out_seg += w coef psi_seg O_B~(p' <- p)^T      (K = dim p)
//   site terms only: out_seg += w coef psi_seg
// The plan cuts every output segment into 32 x 32 tiles and lists, per tile and
// in term order, every contribution reaching it; one workgroup computes one
// tile from its list and writes it once, so the sum has a fixed order and
// needs no atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "rot_internal.h"

namespace rot {
namespace {

constexpr int kSbTile = 32;
constexpr int kSbMaxSite = 16;

enum : int { kFromLeft = 0, kFromRight = 1, kCopy = 2 };

struct SbContrib {
    int kind, K;
    double alpha;
    int64_t a_off, lda;  // left: operator block (rows of the tile); right, copy: psi
    int64_t b_off, ldb;  // left: psi (columns of the tile); right: operator block (rows = tile columns)
};

struct SbTile {
    int64_t out_off, ldo;
    int rows, cols;
    int c_begin, c_end;
};

// C (rows x cols, 32 x 32 at most) = sum of the tile's contributions.  Wave w
// owns the 16 x 16 quarter (w / 2, w % 2) and multiplies with
// v_mfma_f64_16x16x4f64 (lane l supplies A(row l%16, k l/16) and B(k l/16,
// col l%16); accumulator element v is C(4v + l/16, l%16)).  The contributions
// are walked as one sequence of steps (a 32-wide K slice of a product, or a
// scaled copy); the raw operands of the steps one and two ahead are loaded into
// two register sets while the current one is multiplied from LDS (two LDS
// buffers, one barrier per product step), and the step descriptors are read
// from LDS.
constexpr int kSbKs = 32;
constexpr int kSbMaxC = 128;  // contribution descriptors held in LDS at a time

typedef double sb_f64x4 __attribute__((ext_vector_type(4)));

struct SbStep {
    int ci, k0;
};

// Raw operands of step (c, k0) into registers: for a product, this thread's
// four elements of the A slice (tile row r, slice column k) and of the B
// slice; for a copy, the psi entries of this lane's four accumulator rows (in
// av).  Every load is unconditional, from the element's own address when it
// lies inside the slice and from the slice's first element otherwise, and
// nothing is computed from the values here, so the loads stay in flight until
// the step is used; scaling and zeroing happen then (sb_stage, sb_copy).
__device__ __attribute__((always_inline)) inline void sb_load(const SbContrib& c, int k0, const SbTile& tl,
                                                              const double* left_blk, const double* right_blk,
                                                              const double* psi, int tid, int wr, int wc, int h,
                                                              int cl, sb_f64x4& av, sb_f64x4& bv) {
    if (c.kind == kCopy) {
        const int col = wc * 16 + cl, r0 = wr * 16 + h;
        const bool cin = col < tl.cols;
        const double* src = psi + c.a_off;
        av.x = src[(cin && r0 < tl.rows) ? (int64_t)r0 * c.lda + col : 0];
        av.y = src[(cin && r0 + 4 < tl.rows) ? (int64_t)(r0 + 4) * c.lda + col : 0];
        av.z = src[(cin && r0 + 8 < tl.rows) ? (int64_t)(r0 + 8) * c.lda + col : 0];
        av.w = src[(cin && r0 + 12 < tl.rows) ? (int64_t)(r0 + 12) * c.lda + col : 0];
        return;
    }
    const double* A = c.kind == kFromLeft ? left_blk + c.a_off : psi + c.a_off;
    const double* B = c.kind == kFromLeft ? psi + c.b_off : right_blk + c.b_off;
    const bool left = c.kind == kFromLeft;
    // element j of this thread: e = tid + 256 j, A row e >> 5 (col e & 31);
    // B: left, slice row e >> 5 and tile column e & 31; right (B^T stored),
    // tile column e >> 5 and slice row e & 31
    const int hi = tid >> 5, lo = tid & 31;
    double a[4], b[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int r = hi + 8 * j;
        a[j] = A[(r < tl.rows && k0 + lo < c.K) ? (int64_t)r * c.lda + k0 + lo : 0];
        b[j] = B[left ? ((lo < tl.cols && k0 + r < c.K) ? (int64_t)(k0 + r) * c.ldb + lo : 0)
                      : ((r < tl.cols && k0 + lo < c.K) ? (int64_t)r * c.ldb + k0 + lo : 0)];
    }
    av = sb_f64x4{a[0], a[1], a[2], a[3]};
    bv = sb_f64x4{b[0], b[1], b[2], b[3]};
}

// A copy step: alpha times the raw psi entries of this lane's accumulator rows
// (zero outside the tile), as loaded by sb_load.
__device__ __attribute__((always_inline)) inline sb_f64x4 sb_copy(const SbContrib& c, const SbTile& tl,
                                                                  const sb_f64x4& av, int wr, int wc, int h,
                                                                  int cl) {
    const int col = wc * 16 + cl, r0 = wr * 16 + h;
    const bool cin = col < tl.cols;
    return sb_f64x4{(cin && r0 < tl.rows) ? c.alpha * av.x : 0.0, (cin && r0 + 4 < tl.rows) ? c.alpha * av.y : 0.0,
                    (cin && r0 + 8 < tl.rows) ? c.alpha * av.z : 0.0,
                    (cin && r0 + 12 < tl.rows) ? c.alpha * av.w : 0.0};
}

// A product step's slices into LDS: A scaled by alpha, both zero outside the
// slice (the raw values there came from the slice's first element).
__device__ __attribute__((always_inline)) inline void sb_stage(double (*As)[kSbTile + 1], double (*Bs)[kSbTile + 1],
                                                              const SbContrib& c, int k0, const SbTile& tl,
                                                              const sb_f64x4& av, const sb_f64x4& bv, int tid) {
    const int hi = tid >> 5, lo = tid & 31;
    const bool left = c.kind == kFromLeft;
    const double a[4] = {av.x, av.y, av.z, av.w}, b[4] = {bv.x, bv.y, bv.z, bv.w};
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int r = hi + 8 * j;
        As[lo][r] = (r < tl.rows && k0 + lo < c.K) ? c.alpha * a[j] : 0.0;
        if (left)
            Bs[r][lo] = (lo < tl.cols && k0 + r < c.K) ? b[j] : 0.0;
        else
            Bs[lo][r] = (r < tl.cols && k0 + lo < c.K) ? b[j] : 0.0;
    }
}

// position after step x of the chunk [.., ce) whose descriptors start at cd[0] (index cb)
__device__ __attribute__((always_inline)) inline SbStep sb_next(const SbContrib* cd, int cb, int ce, SbStep x) {
    if (x.ci >= ce) return x;
    const SbContrib& c = cd[x.ci - cb];
    return (c.kind == kCopy || x.k0 + kSbKs >= c.K) ? SbStep{x.ci + 1, 0} : SbStep{x.ci, x.k0 + kSbKs};
}

__global__ __launch_bounds__(256) void sb_tile_kernel(const SbTile* __restrict__ tiles,
                                                      const SbContrib* __restrict__ contribs,
                                                      const double* __restrict__ left_blk,
                                                      const double* __restrict__ right_blk,
                                                      const double* __restrict__ psi, double* __restrict__ out) {
    const SbTile tl = tiles[blockIdx.x];
    __shared__ double As[2][kSbKs][kSbTile + 1];  // [buf][k][row]
    __shared__ double Bs[2][kSbKs][kSbTile + 1];  // [buf][k][col]
    __shared__ SbContrib cd[kSbMaxC];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1, h = lane >> 4, cl = lane & 15;
    sb_f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    sb_f64x4 a0, b0, a1, b1;
    int buf = 0;
// one step from register set (A, B); the set is then refilled with step REFILL
#define SB_RUN(A, B, X, REFILL)                                                                            \
    do {                                                                                                      \
        const SbContrib& c_ = cd[(X).ci - cb];                                                                \
        if (c_.kind == kCopy) {                                                                               \
            acc += sb_copy(c_, tl, A, wr, wc, h, cl);                                                         \
            if ((REFILL).ci < ce)                                                                             \
                sb_load(cd[(REFILL).ci - cb], (REFILL).k0, tl, left_blk, right_blk, psi, tid, wr, wc, h, cl, A, \
                        B);                                                                                \
        } else {                                                                                              \
            sb_stage(As[buf], Bs[buf], c_, (X).k0, tl, A, B, tid);                                            \
            __syncthreads();                                                                                  \
            const int kq = (min(kSbKs, c_.K - (X).k0) + 3) >> 2;                                              \
            if ((REFILL).ci < ce)                                                                             \
                sb_load(cd[(REFILL).ci - cb], (REFILL).k0, tl, left_blk, right_blk, psi, tid, wr, wc, h, cl, A, \
                        B);                                                                                \
            for (int q = 0; q < kq; q++) {                                                                    \
                const double a_ = As[buf][4 * q + h][wr * 16 + cl];                                           \
                const double b_ = Bs[buf][4 * q + h][wc * 16 + cl];                                           \
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a_, b_, acc, 0, 0, 0);                             \
            }                                                                                                 \
            buf ^= 1;                                                                                         \
        }                                                                                                     \
    } while (0)
    for (int cb = tl.c_begin; cb < tl.c_end; cb += kSbMaxC) {
        const int ce = min(cb + kSbMaxC, tl.c_end);
        __syncthreads();  // the previous chunk's descriptors are no longer read
        for (int i = tid; i < ce - cb; i += 256) cd[i] = contribs[cb + i];
        __syncthreads();
        SbStep cur{cb, 0};
        SbStep s1 = sb_next(cd, cb, ce, cur);
        sb_load(cd[0], 0, tl, left_blk, right_blk, psi, tid, wr, wc, h, cl, a0, b0);
        if (s1.ci < ce) sb_load(cd[s1.ci - cb], s1.k0, tl, left_blk, right_blk, psi, tid, wr, wc, h, cl, a1, b1);
        SbStep ld = sb_next(cd, cb, ce, s1);
        while (true) {
            SB_RUN(a0, b0, cur, ld);
            cur = sb_next(cd, cb, ce, cur);
            ld = sb_next(cd, cb, ce, ld);
            if (cur.ci >= ce) break;
            SB_RUN(a1, b1, cur, ld);
            cur = sb_next(cd, cb, ce, cur);
            ld = sb_next(cd, cb, ce, ld);
            if (cur.ci >= ce) break;
        }
    }
#undef SB_RUN
#pragma unroll
    for (int v = 0; v < 4; v++) {
        const int r = wr * 16 + 4 * v + h, col = wc * 16 + cl;
        if (r < tl.rows && col < tl.cols) out[tl.out_off + r * tl.ldo + col] = acc[v];
    }
}

rot_status sberr(rot_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return set_error(s, buf);
}

using Qn = std::pair<int, int>;

// One segment of a system (or environment) sector: site state, block sector
// index and its first row (column) inside the sector.
struct Seg {
    int site, sec, start, dim;
};

struct Enlarged {
    std::map<Qn, std::vector<Seg>> segs;  // by sector numbers, segments in site order
    std::map<Qn, int> dim;
};

Enlarged enlarge(int d, const int32_t* site_qn, int n_sec, const rot_sector* sec) {
    Enlarged E;
    std::map<Qn, int> by_qn;
    for (int k = 0; k < n_sec; k++) by_qn[{sec[k].n_up, sec[k].n_dn}] = k;
    std::map<Qn, bool> seen;
    for (int k = 0; k < n_sec; k++)
        for (int s = 0; s < d; s++) seen[{sec[k].n_up + site_qn[2 * s], sec[k].n_dn + site_qn[2 * s + 1]}] = true;
    for (auto& kv : seen) {
        const Qn Q = kv.first;
        int start = 0;
        std::vector<Seg> v;
        for (int s = 0; s < d; s++) {
            auto it = by_qn.find({Q.first - site_qn[2 * s], Q.second - site_qn[2 * s + 1]});
            if (it == by_qn.end()) continue;
            v.push_back({s, it->second, start, sec[it->second].dim});
            start += sec[it->second].dim;
        }
        E.segs[Q] = v;
        E.dim[Q] = start;
    }
    return E;
}

struct Block {
    Qn Q;
    int rows, cols;
    int64_t offset;
};

std::vector<Block> psi_blocks(const rot_sb_problem* p, const Enlarged& sys, const Enlarged& env) {
    std::vector<Block> out;
    int64_t off = 0;
    for (auto& kv : sys.dim) {
        const Qn P{p->target[0] - kv.first.first, p->target[1] - kv.first.second};
        auto it = env.dim.find(P);
        if (it == env.dim.end()) continue;
        out.push_back({kv.first, kv.second, it->second, off});
        off += (int64_t)kv.second * it->second;
    }
    return out;
}

rot_status validate_sb(const rot_sb_problem* p) {
    if (!p) return sberr(ROT_ERR_INVALID_ARG, "null problem");
    if (p->d < 1 || p->d > kSbMaxSite || !p->site_qn) return sberr(ROT_ERR_INVALID_ARG, "need 1 <= d <= %d and site_qn", kSbMaxSite);
    for (int side = 0; side < 2; side++) {
        const int n = side ? p->n_right : p->n_left;
        const rot_sector* sec = side ? p->right : p->left;
        if (n < 1 || !sec) return sberr(ROT_ERR_INVALID_ARG, "%s block: need at least one sector", side ? "right" : "left");
        std::map<Qn, int> seen;
        for (int k = 0; k < n; k++) {
            if (sec[k].dim < 1) return sberr(ROT_ERR_INVALID_ARG, "%s sector %d: dim < 1", side ? "right" : "left", k);
            if (seen.count({sec[k].n_up, sec[k].n_dn}))
                return sberr(ROT_ERR_INVALID_ARG, "%s sector %d: repeated numbers", side ? "right" : "left", k);
            seen[{sec[k].n_up, sec[k].n_dn}] = k;
        }
        const int n_ops = side ? p->n_right_ops : p->n_left_ops;
        if (n_ops < 0) return sberr(ROT_ERR_INVALID_ARG, "negative operator count");
        if (n_ops > 0) {
            const int32_t* sh = side ? p->right_shift : p->left_shift;
            const int64_t* off = side ? p->right_off : p->left_off;
            const double* blk = side ? p->right_blk : p->left_blk;
            if (!sh || !off) return sberr(ROT_ERR_INVALID_ARG, "%s operators: null shift or offset table", side ? "right" : "left");
            bool any = false;
            for (int64_t e = 0; e < (int64_t)n_ops * n; e++) {
                if (off[e] < -1) return sberr(ROT_ERR_INVALID_ARG, "operator offset below -1");
                any = any || off[e] >= 0;
            }
            if (any && !blk) return sberr(ROT_ERR_INVALID_ARG, "%s operators: null block data", side ? "right" : "left");
        }
    }
    if (p->n_terms < 0 || (p->n_terms > 0 && !p->terms)) return sberr(ROT_ERR_INVALID_ARG, "null terms");
    for (int l = 0; l < p->n_terms; l++) {
        const rot_sb_term& t = p->terms[l];
        if (t.left_op < -1 || t.left_op >= p->n_left_ops || t.right_op < -1 || t.right_op >= p->n_right_ops)
            return sberr(ROT_ERR_INVALID_ARG, "term %d: operator index out of range", l);
        if (t.left_op >= 0 && t.right_op >= 0)
            return sberr(ROT_ERR_UNSUPPORTED, "term %d: operators on both blocks are not supported", l);
        int dn[2] = {0, 0};
        if (t.left_op >= 0) {
            dn[0] += p->left_shift[2 * t.left_op];
            dn[1] += p->left_shift[2 * t.left_op + 1];
        }
        if (t.right_op >= 0) {
            dn[0] += p->right_shift[2 * t.right_op];
            dn[1] += p->right_shift[2 * t.right_op + 1];
        }
        for (int w = 0; w < 2; w++) {
            const double* S = w ? t.site_at : t.site_a;
            if (!S) continue;
            bool have = false;
            int sh[2] = {0, 0};
            for (int a = 0; a < p->d; a++)
                for (int b = 0; b < p->d; b++) {
                    if (S[a * p->d + b] == 0.0) continue;
                    const int x = p->site_qn[2 * a] - p->site_qn[2 * b], y = p->site_qn[2 * a + 1] - p->site_qn[2 * b + 1];
                    if (have && (x != sh[0] || y != sh[1]))
                        return sberr(ROT_ERR_INVALID_ARG, "term %d: site matrix mixes particle-number shifts", l);
                    have = true;
                    sh[0] = x;
                    sh[1] = y;
                }
            dn[0] += sh[0];
            dn[1] += sh[1];
        }
        if (dn[0] != 0 || dn[1] != 0) return sberr(ROT_ERR_INVALID_ARG, "term %d: shifts do not add to zero", l);
    }
    return ROT_OK;
}

// Output tiles and their contributions, in block, segment, tile and then term
// order (site states of the term's sums in ascending order).
void build_work(const rot_sb_problem* p, std::vector<SbTile>& tiles, std::vector<SbContrib>& cs, double& flops,
                int64_t& total) {
    const Enlarged sys = enlarge(p->d, p->site_qn, p->n_left, p->left);
    const Enlarged env = enlarge(p->d, p->site_qn, p->n_right, p->right);
    const std::vector<Block> blocks = psi_blocks(p, sys, env);
    total = blocks.empty() ? 0 : blocks.back().offset + (int64_t)blocks.back().rows * blocks.back().cols;
    std::map<Qn, const Block*> block_of;
    for (const Block& b : blocks) block_of[b.Q] = &b;
    std::map<Qn, int> lsec, rsec;
    for (int k = 0; k < p->n_left; k++) lsec[{p->left[k].n_up, p->left[k].n_dn}] = k;
    for (int k = 0; k < p->n_right; k++) rsec[{p->right[k].n_up, p->right[k].n_dn}] = k;
    // first row (column) of segment (site state, block sector) inside an enlarged sector
    auto seg_start = [](const Enlarged& E, Qn Q, int site, int sec) {
        auto it = E.segs.find(Q);
        if (it == E.segs.end()) return -1;
        for (const Seg& g : it->second)
            if (g.site == site && g.sec == sec) return g.start;
        return -1;
    };
    const int d = p->d;
    const int32_t* qn = p->site_qn;
    flops = 0.0;
    for (const Block& ob : blocks) {
        const Qn P{p->target[0] - ob.Q.first, p->target[1] - ob.Q.second};
        for (const Seg& rs : sys.segs.at(ob.Q)) {
            const Qn qo{p->left[rs.sec].n_up, p->left[rs.sec].n_dn};
            for (const Seg& csg : env.segs.at(P)) {
                const Qn po{p->right[csg.sec].n_up, p->right[csg.sec].n_dn};
                for (int r0 = 0; r0 < rs.dim; r0 += kSbTile)
                    for (int c0 = 0; c0 < csg.dim; c0 += kSbTile) {
                        SbTile tl{};
                        tl.out_off = ob.offset + (int64_t)(rs.start + r0) * ob.cols + csg.start + c0;
                        tl.ldo = ob.cols;
                        tl.rows = std::min(kSbTile, rs.dim - r0);
                        tl.cols = std::min(kSbTile, csg.dim - c0);
                        tl.c_begin = (int)cs.size();
                        for (int l = 0; l < p->n_terms; l++) {
                            const rot_sb_term& t = p->terms[l];
                            const int lo = t.left_op, ro = t.right_op;
                            const Qn qs{qo.first - (lo >= 0 ? p->left_shift[2 * lo] : 0),
                                        qo.second - (lo >= 0 ? p->left_shift[2 * lo + 1] : 0)};
                            const Qn ps{po.first - (ro >= 0 ? p->right_shift[2 * ro] : 0),
                                        po.second - (ro >= 0 ? p->right_shift[2 * ro + 1] : 0)};
                            auto kq = lsec.find(qs);
                            auto kp = rsec.find(ps);
                            if (kq == lsec.end() || kp == rsec.end()) continue;
                            int64_t op_off = -1;
                            if (lo >= 0) op_off = p->left_off[(int64_t)lo * p->n_left + kq->second];
                            if (ro >= 0) op_off = p->right_off[(int64_t)ro * p->n_right + kp->second];
                            if ((lo >= 0 || ro >= 0) && op_off < 0) continue;
                            for (int sa = 0; sa < d; sa++) {
                                const double wa = t.site_a ? t.site_a[rs.site * d + sa] : (sa == rs.site ? 1.0 : 0.0);
                                if (wa == 0.0) continue;
                                for (int ta = 0; ta < d; ta++) {
                                    const double wt = t.site_at ? t.site_at[csg.site * d + ta] : (ta == csg.site ? 1.0 : 0.0);
                                    if (wt == 0.0) continue;
                                    const Qn Qs{qs.first + qn[2 * sa], qs.second + qn[2 * sa + 1]};
                                    const Qn Ps{ps.first + qn[2 * ta], ps.second + qn[2 * ta + 1]};
                                    auto sb = block_of.find(Qs);
                                    if (sb == block_of.end()) continue;
                                    const Block& src = *sb->second;
                                    const int rstart = seg_start(sys, Qs, sa, kq->second);
                                    const int cstart = seg_start(env, Ps, ta, kp->second);
                                    if (rstart < 0 || cstart < 0) continue;
                                    SbContrib c{};
                                    c.alpha = t.coef * wa * wt;
                                    if (lo >= 0) {
                                        const int K = p->left[kq->second].dim;
                                        c.kind = kFromLeft;
                                        c.K = K;
                                        c.a_off = op_off + (int64_t)r0 * K;
                                        c.lda = K;
                                        c.b_off = src.offset + (int64_t)rstart * src.cols + cstart + c0;
                                        c.ldb = src.cols;
                                    } else if (ro >= 0) {
                                        const int K = p->right[kp->second].dim;
                                        c.kind = kFromRight;
                                        c.K = K;
                                        c.a_off = src.offset + (int64_t)(rstart + r0) * src.cols + cstart;
                                        c.lda = src.cols;
                                        c.b_off = op_off + (int64_t)c0 * K;
                                        c.ldb = K;
                                    } else {
                                        c.kind = kCopy;
                                        c.K = 1;
                                        c.a_off = src.offset + (int64_t)(rstart + r0) * src.cols + cstart + c0;
                                        c.lda = src.cols;
                                    }
                                    flops += 2.0 * tl.rows * tl.cols * c.K;
                                    cs.push_back(c);
                                }
                            }
                        }
                        tl.c_end = (int)cs.size();
                        tiles.push_back(tl);
                    }
            }
        }
    }
}

}  // namespace
}  // namespace rot

struct rot_sb_plan_s {
    rot::SbTile* tiles = nullptr;
    rot::SbContrib* contribs = nullptr;
    int n_tiles = 0;
    const double* left_blk = nullptr;
    const double* right_blk = nullptr;
    int64_t total = 0;
    double flops = 0.0;
};

using namespace rot;

extern "C" {

rot_status rot_sb_layout(const rot_sb_problem* p, int32_t capacity, int32_t* n_blocks, int32_t* qn, int32_t* rows,
                         int32_t* cols, int64_t* offset, int64_t* total) {
    const rot_status v = validate_sb(p);
    if (v != ROT_OK) return v;
    if (!n_blocks || !total) return sberr(ROT_ERR_INVALID_ARG, "null n_blocks or total");
    const Enlarged sys = enlarge(p->d, p->site_qn, p->n_left, p->left);
    const Enlarged env = enlarge(p->d, p->site_qn, p->n_right, p->right);
    const std::vector<Block> blocks = psi_blocks(p, sys, env);
    *n_blocks = (int32_t)blocks.size();
    *total = blocks.empty() ? 0 : blocks.back().offset + (int64_t)blocks.back().rows * blocks.back().cols;
    const int n = std::min<int>(std::max(capacity, 0), (int)blocks.size());
    for (int k = 0; k < n; k++) {
        if (qn) {
            qn[2 * k] = blocks[k].Q.first;
            qn[2 * k + 1] = blocks[k].Q.second;
        }
        if (rows) rows[k] = blocks[k].rows;
        if (cols) cols[k] = blocks[k].cols;
        if (offset) offset[k] = blocks[k].offset;
    }
    return ROT_OK;
}

rot_status rot_sb_plan_create(const rot_sb_problem* p, rot_sb_plan* plan) {
    rot::TraceRange trace_("rot_sb_plan_create");
    if (!plan) return sberr(ROT_ERR_INVALID_ARG, "null plan output");
    *plan = nullptr;
    const rot_status v = validate_sb(p);
    if (v != ROT_OK) return v;
    std::vector<SbTile> tiles;
    std::vector<SbContrib> cs;
    auto* P = new rot_sb_plan_s();
    build_work(p, tiles, cs, P->flops, P->total);
    // heaviest tiles first: all tiles do not fit on the chip at once, and the
    // ones dispatched last should be short
    {
        std::vector<std::pair<int64_t, int>> order(tiles.size());
        for (size_t i = 0; i < tiles.size(); i++) {
            int64_t w = 0;
            for (int c = tiles[i].c_begin; c < tiles[i].c_end; c++) w += cs[c].kind == kCopy ? 1 : (cs[c].K + 31) / 32;
            order[i] = {-w, (int)i};
        }
        std::stable_sort(order.begin(), order.end());
        std::vector<SbTile> sorted(tiles.size());
        for (size_t i = 0; i < tiles.size(); i++) sorted[i] = tiles[order[i].second];
        tiles.swap(sorted);
    }
    P->n_tiles = (int)tiles.size();
    P->left_blk = p->left_blk;
    P->right_blk = p->right_blk;
    hipError_t e = hipSuccess;
    if (!tiles.empty()) {
        e = hipMalloc(&P->tiles, sizeof(SbTile) * tiles.size());
        if (e == hipSuccess) e = hipMalloc(&P->contribs, sizeof(SbContrib) * std::max<size_t>(cs.size(), 1));
        if (e == hipSuccess) e = hipMemcpy(P->tiles, tiles.data(), sizeof(SbTile) * tiles.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess && !cs.empty())
            e = hipMemcpy(P->contribs, cs.data(), sizeof(SbContrib) * cs.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        rot_sb_plan_destroy(P);
        return sberr(ROT_ERR_HIP, "rot_sb_plan_create: %s", hipGetErrorString(e));
    }
    *plan = P;
    return ROT_OK;
}

rot_status rot_sb_apply(rot_sb_plan plan, const double* psi, double* out, void* stream) {
    rot::TraceRange trace_("rot_sb_apply");
    if (!plan) return sberr(ROT_ERR_INVALID_ARG, "null plan");
    if (plan->total == 0) return ROT_OK;
    if (!psi || !out) return sberr(ROT_ERR_INVALID_ARG, "null psi or out");
    if (out < psi + plan->total && psi < out + plan->total) return sberr(ROT_ERR_INVALID_ARG, "out overlaps psi");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hipError_t e = prof_timed("sb_matvec", s, [&] {
        hipLaunchKernelGGL(sb_tile_kernel, dim3(plan->n_tiles), dim3(256), 0, s, plan->tiles, plan->contribs,
                           plan->left_blk, plan->right_blk, psi, out);
        return hipGetLastError();
    });
    return e == hipSuccess ? ROT_OK : sberr(ROT_ERR_HIP, "rot_sb_apply: %s", hipGetErrorString(e));
}

double rot_sb_plan_flops(rot_sb_plan plan) { return plan ? plan->flops : 0.0; }

rot_status rot_sb_plan_destroy(rot_sb_plan plan) {
    if (!plan) return ROT_OK;
    if (plan->tiles) (void)hipFree(plan->tiles);
    if (plan->contribs) (void)hipFree(plan->contribs);
    delete plan;
    return ROT_OK;
}

}  // extern "C"
