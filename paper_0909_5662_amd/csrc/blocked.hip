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
#include <cstring>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "rot_internal.h"

namespace rot {
namespace {

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
    std::vector<unsigned char> sig;
    DeviceLists s1, s2;
    int* counter = nullptr;
    int64_t x_elems = 0;
    ~Plan() {
        (void)hipFree(s1.probs);
        (void)hipFree(s1.tiles);
        (void)hipFree(s2.probs);
        (void)hipFree(s2.tiles);
        (void)hipFree(counter);
    }
};

std::mutex g_mu;
std::list<std::unique_ptr<Plan>> g_plans;  // most recent first

template <class T>
void put(std::vector<unsigned char>& v, const T* p, size_t n) {
    const unsigned char* c = reinterpret_cast<const unsigned char*>(p);
    v.insert(v.end(), c, c + sizeof(T) * n);
}

// Everything the work-lists depend on: the tables' contents, the shape, and
// the 16-byte alignment of the buffers (which decides vector loads).
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

}  // namespace

size_t blocked_workspace_bytes(const rot_blocked_problem* p) {
    Structure st;
    std::string why;
    if (!build_structure(p, &st, &why)) return 0;
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
    return (size_t)x * sizeof(float);
}

rot_status blocked_validate(const rot_blocked_problem* p, std::string* why) {
    Structure st;
    return build_structure(p, &st, why) ? ROT_OK : ROT_ERR_INVALID_ARG;
}

hipError_t rotate_blocked(const rot_blocked_problem* p, void* ws, size_t ws_bytes, hipStream_t stream) {
    (void)ws_bytes;
    if (p->n_ops == 0) return hipSuccess;
    const GroupedShape shape = blocked_shape();
    std::vector<unsigned char> sig = signature(p, ws, shape);
    Plan* plan = nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto it = g_plans.begin(); it != g_plans.end(); ++it) {
        if ((*it)->sig == sig) {
            g_plans.splice(g_plans.begin(), g_plans, it);
            plan = g_plans.front().get();
            break;
        }
    }
    if (!plan) {
        Structure st;
        std::string why;
        if (!build_structure(p, &st, &why)) return hipErrorInvalidValue;  // validated by the caller
        Lists L;
        build_lists(p, st, static_cast<const float*>(ws), &L);
        auto np = std::make_unique<Plan>();
        np->sig = std::move(sig);
        np->x_elems = L.x_elems;
        const int edge = grouped_tile_edge(shape);
        hipError_t e = upload(L.p1, make_tiles(L.p1, edge), &np->s1);
        if (e == hipSuccess) e = upload(L.p2, make_tiles(L.p2, edge), &np->s2);
        if (e == hipSuccess) e = hipMalloc(&np->counter, sizeof(int));
        if (e != hipSuccess) return e;
        g_plans.push_front(std::move(np));
        if (g_plans.size() > kPlanCacheSize) g_plans.pop_back();
        plan = g_plans.front().get();
    }
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
    a.counter = plan->counter;
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

}  // namespace rot
