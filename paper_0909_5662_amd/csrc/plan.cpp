// Plans: repeated rotation of a fixed set of groups of different sizes (one
// DMRG sweep step rotates the stored operators of many blocks), executed as
// grouped persistent launches captured in one hipGraph.
//
// rot_plan_create
//   1. buckets groups into size classes (ceil log2 of m*d and of m'),
//   2. packs each class's operators into chunks whose stage-1 intermediates
//      fit the workspace (largest classes first),
//   3. builds per-chunk work-lists (one problem per operator and stage, tiles
//      in longest-processing-time order) in plan-owned device memory,
//   4. picks, per class, the tile shape and the schedule (static contiguous
//      runs, the uniform-matrix distribution of Sec. 3.2, or an atomic tile
//      queue, the pool of tasks of Sec. 3.2) from the tuning cache, timing the
//      candidates on the class's first chunk when the cache has no entry,
//   5. captures every launch, in order, into a hipGraph on a plan-owned stream.
// rot_plan_execute replays the graph on the caller's stream (or re-issues the
// launches when graphs are disabled).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "rot_internal.h"

struct rot_plan_s {
    struct Launch {
        int cls;
        int stage;  // 1 or 2
        rot::GroupedProblem* probs = nullptr;
        rot::GroupedTile* tiles = nullptr;
        int n_tiles = 0;
        int* counter = nullptr;
        double flops = 0;
        std::vector<std::pair<int, int>> src;  // (group, operator) of each problem
        std::vector<const float*> t;           // its stage-1 intermediate
    };
    struct Class {
        std::string key;
        rot::GroupedShape shape = rot::GroupedShape::k128;
        bool dynamic = true;
        int grid = 0;
        bool tuned = false;
        double flops = 0;
        int n_ops = 0;
    };
    std::vector<Class> classes;
    std::vector<Launch> launches;
    std::vector<std::vector<rot::GroupedProblem>> host_probs;  // per launch (tiles rebuilt on shape change)
    std::vector<rot_problem> groups;  // resolved shapes and the bound buffers
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool use_graph = true;
    // rot_plan_rebind: pinned staging of the problem tables and the event of
    // the last copy out of it
    rot::GroupedProblem* staging = nullptr;
    size_t staging_count = 0;
    hipEvent_t staged = nullptr;
    std::string error;
};

namespace rot {
namespace {

rot_status perr(rot_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return set_error(s, buf);
}

int ceil_log2(int64_t x) {
    int k = 0;
    while ((int64_t(1) << k) < x) k++;
    return k;
}

// ---------------------------------------------------------------- tuning --
const char* shape_name(GroupedShape s) {
    return s == GroupedShape::k128d ? "128d" : s == GroupedShape::k128 ? "128" : s == GroupedShape::k64 ? "64" : "32";
}

// A plan class's cached choice: tokens "tile-edge schedule persistent-grid"
// (tile edge 128d: 128 with K slices copied straight into LDS);
// false when absent or not of that form.
bool cached_choice(const std::string& key, GroupedShape* shape, bool* dynamic, int* grid) {
    std::vector<std::string> t;
    if (!tune_get(key, &t) || t.size() != 3) return false;
    if (t[0] != "128" && t[0] != "128d" && t[0] != "64" && t[0] != "32") return false;
    if (t[1] != "static" && t[1] != "dynamic") return false;
    char* end = nullptr;
    const long g = strtol(t[2].c_str(), &end, 10);
    if (!end || *end || g < 0 || g > (1 << 24)) return false;
    *shape = t[0] == "64"     ? GroupedShape::k64
             : t[0] == "32"   ? GroupedShape::k32
             : t[0] == "128d" ? GroupedShape::k128d
                              : GroupedShape::k128;
    *dynamic = t[1] == "dynamic";
    *grid = (int)g;
    return true;
}

// The grouped-GEMM problem of stage 1 or 2 for operator b of group p (p
// resolved), with T its stage-1 intermediate.  Positions are absolute
// addresses (the launches' base pointers are null).  T_b takes U's row
// layout ((m*d) x ldu): stage 1 reads U_r as one matrix of row stride d*ldu
// over (d-1)*ldu + mp columns.
GroupedProblem stage_problem(const rot_problem& p, int b, const float* T, int stage) {
    const float* O = static_cast<const float*>(p.O) + (int64_t)b * p.stride_o;
    float* out = static_cast<float*>(p.out) + (int64_t)b * p.stride_out;
    const float* U = static_cast<const float*>(p.U);
    auto al = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
    auto addr = [](const void* q) { return (int64_t) reinterpret_cast<uintptr_t>(q); };
    GroupedProblem g{};
    if (stage == 1) {
        g.M = p.m;
        g.N = (int)((int64_t)(p.d - 1) * p.ldu + p.mp);
        g.K = p.m;
        g.a_off = addr(O);
        g.lda = p.ldo;
        g.b_off = addr(U);
        g.ldb = (int64_t)p.d * p.ldu;
        g.c_off = addr(T);
        g.ldc = (int64_t)p.d * p.ldu;
        g.flags = (al(O) && al(U) && p.ldo % 4 == 0 && (p.d * p.ldu) % 4 == 0) ? kGroupedVec : 0;
    } else {
        g.M = p.mp;
        g.N = p.mp;
        g.K = p.m * p.d;
        g.a_off = addr(U);
        g.lda = p.ldu;
        g.b_off = addr(T);
        g.ldb = p.ldu;
        g.c_off = addr(out);
        g.ldc = p.ldout;
        g.flags = (al(U) && p.ldu % 4 == 0) ? kGroupedVec : 0;
    }
    // whole tiles and slices for buffer loads with LDS destination (A is
    // K-contiguous in stage 1, M-contiguous in stage 2; B is N-contiguous)
    const int64_t ea = stage == 1 ? (int64_t)(g.M - 1) * g.lda + g.K : (int64_t)(g.K - 1) * g.lda + g.M;
    const int64_t eb = (int64_t)(g.K - 1) * g.ldb + g.N;
    if ((g.flags & kGroupedVec) && g.M % 128 == 0 && g.N % 128 == 0 && g.K % 16 == 0 && g.K > 0 &&
        ea * 4 < ((int64_t)1 << 32) && eb * 4 < ((int64_t)1 << 32))
        g.flags |= kGroupedWhole;
    return g;
}

// Every problem of class `ci`'s launches is whole (the k128d shape applies).
bool class_whole(const rot_plan_s* P, int ci) {
    for (size_t li = 0; li < P->launches.size(); li++) {
        if (P->launches[li].cls != ci) continue;
        for (const GroupedProblem& g : P->host_probs[li])
            if (!(g.flags & kGroupedWhole)) return false;
    }
    return true;
}

std::vector<GroupedTile> tiles_for(const std::vector<GroupedProblem>& probs, int edge) {
    std::vector<GroupedTile> t;
    for (int i = 0; i < (int)probs.size(); i++)
        for (int n0 = 0; n0 < probs[i].N; n0 += edge)
            for (int m0 = 0; m0 < probs[i].M; m0 += edge) t.push_back(GroupedTile{i, m0, n0, 0});
    std::stable_sort(t.begin(), t.end(),
                     [&](const GroupedTile& a, const GroupedTile& b) { return probs[a.prob].K > probs[b.prob].K; });
    return t;
}

hipError_t upload_tiles(rot_plan_s::Launch& L, const std::vector<GroupedProblem>& probs, GroupedShape shape) {
    std::vector<GroupedTile> t = tiles_for(probs, grouped_tile_edge(shape));
    if (L.tiles) (void)hipFree(L.tiles);
    L.tiles = nullptr;
    L.n_tiles = (int)t.size();
    hipError_t e = hipMalloc(&L.tiles, sizeof(GroupedTile) * t.size());
    if (e == hipSuccess) e = hipMemcpy(L.tiles, t.data(), sizeof(GroupedTile) * t.size(), hipMemcpyHostToDevice);
    return e;
}

GroupedLaunch make_launch(const rot_plan_s::Launch& L, const rot_plan_s::Class& c) {
    GroupedLaunch g{};
    g.a_base = nullptr;
    g.b_base = nullptr;
    g.c_base = nullptr;
    g.probs = L.probs;
    g.tiles = L.tiles;
    g.n_tiles = L.n_tiles;
    g.a_kcontig = L.stage == 1;  // stage 1: A = O_b (K-contiguous); stage 2: A = U^T view
    g.b_kcontig = false;
    g.dynamic = c.dynamic;
    g.shape = c.shape;
    g.grid = c.grid;
    g.counter = L.counter;
    return g;
}

// Enqueue every launch of the plan; `timed` files each under the profiler
// (never while capturing).
hipError_t issue_all(rot_plan_s* P, hipStream_t s, bool timed) {
    for (auto& L : P->launches) {
        const GroupedLaunch g = make_launch(L, P->classes[L.cls]);
        const char* name = L.stage == 1 ? "plan_stage1_fp32" : "plan_stage2_fp32";
        hipError_t e = timed ? prof_timed(name, s, [&] { return grouped_gemm_f32(g, s); }) : grouped_gemm_f32(g, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Time the candidates for class `ci` on its first chunk (both stages).
hipError_t tune_class(rot_plan_s* P, int ci, int n_cu) {
    rot_plan_s::Class& c = P->classes[ci];
    int l1 = -1, l2 = -1;
    for (int i = 0; i < (int)P->launches.size(); i++)
        if (P->launches[i].cls == ci) {
            if (P->launches[i].stage == 1 && l1 < 0) l1 = i;
            if (P->launches[i].stage == 2 && l2 < 0 && l1 >= 0) l2 = i;
        }
    if (l1 < 0 || l2 < 0) return hipSuccess;
    struct Cand {
        GroupedShape shape;
        bool dynamic;
        int grid_per_cu;  // 0: one workgroup per tile
    };
    // 128 x 128 tiles run at up to 3 workgroups (12 waves) per CU, 64 x 64 at
    // 7, 128 x 128 with slices by buffer loads with LDS destination (whole
    // problems only) at 4
    const bool whole = class_whole(P, ci);
    const Cand all[] = {
        {GroupedShape::k128, false, 0},  {GroupedShape::k128, true, 2},   {GroupedShape::k128, false, 2},
        {GroupedShape::k128, true, 3},   {GroupedShape::k128, false, 3},  {GroupedShape::k64, false, 0},
        {GroupedShape::k64, true, 6},    {GroupedShape::k128d, false, 0}, {GroupedShape::k128d, true, 4},
        {GroupedShape::k128d, false, 4},
    };
    std::vector<Cand> cands;
    for (const Cand& cd : all)
        if (cd.shape != GroupedShape::k128d || whole) cands.push_back(cd);
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e != hipSuccess) return e;
    float best = 1e30f;
    Cand best_c = cands[0];
    for (const Cand& cd : cands) {
        c.shape = cd.shape;
        c.dynamic = cd.dynamic;
        c.grid = cd.grid_per_cu * n_cu;
        for (int li : {l1, l2}) {
            e = upload_tiles(P->launches[li], P->host_probs[li], cd.shape);
            if (e != hipSuccess) break;
        }
        if (e != hipSuccess) break;
        float total = 0.f;
        for (int rep = 0; rep < 3 && e == hipSuccess; rep++) {
            e = hipEventRecord(a, P->stream);
            for (int li : {l1, l2}) {
                if (e != hipSuccess) break;
                e = grouped_gemm_f32(make_launch(P->launches[li], c), P->stream);
            }
            if (e == hipSuccess) e = hipEventRecord(b, P->stream);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            if (rep > 0) total += ms;  // first run warms up
        }
        if (e != hipSuccess) break;
        if (total < best) {
            best = total;
            best_c = cd;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return e;
    c.shape = best_c.shape;
    c.dynamic = best_c.dynamic;
    c.grid = best_c.grid_per_cu * n_cu;
    c.tuned = true;
    return hipSuccess;
}

void destroy(rot_plan_s* P) {
    if (!P) return;
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    for (auto& L : P->launches) {
        (void)hipFree(L.probs);
        (void)hipFree(L.tiles);
        (void)hipFree(L.counter);
    }
    if (P->staged) {
        (void)hipEventSynchronize(P->staged);
        (void)hipEventDestroy(P->staged);
    }
    if (P->staging) (void)hipHostFree(P->staging);
    if (P->stream) (void)hipStreamDestroy(P->stream);
    delete P;
}

}  // namespace
}  // namespace rot

using namespace rot;

extern "C" {

rot_status rot_plan_create(const rot_problem* groups, int32_t n_groups, rot_precision prec, void* workspace,
                           size_t workspace_bytes, uint32_t flags, void* stream, rot_plan* out) {
    rot::TraceRange trace_("rot_plan_create");
    if (!out) return perr(ROT_ERR_INVALID_ARG, "null plan output");
    *out = nullptr;
    if (n_groups < 0 || (n_groups > 0 && !groups)) return perr(ROT_ERR_INVALID_ARG, "null groups or n_groups < 0");
    if (prec != ROT_FP32) return perr(ROT_ERR_UNSUPPORTED, "plans support ROT_FP32 only");
    if (flags & ~(ROT_PLAN_NO_GRAPH | ROT_PLAN_NO_TUNE | ROT_PLAN_RETUNE))
        return perr(ROT_ERR_INVALID_ARG, "unknown plan flags 0x%x", flags);
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return perr(ROT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    // validation (same rules as rot_batch); leading dimensions 0 select the packed values
    std::vector<rot_problem> rg(groups, groups + n_groups);
    size_t min_ws = 0;
    for (int gi = 0; gi < n_groups; gi++) {
        rot_problem& p = rg[gi];
        if (p.ldu == 0) p.ldu = p.mp;
        if (p.ldo == 0) p.ldo = p.m;
        if (p.ldout == 0) p.ldout = p.mp;
        if (p.m <= 0 || p.d <= 0 || p.mp <= 0 || p.n_ops < 0 || (int64_t)p.m * p.d > INT32_MAX ||
            (int64_t)p.d * p.mp > INT32_MAX || p.mp > (int64_t)p.m * p.d)
            return perr(ROT_ERR_INVALID_ARG, "group %d: need m, d, mp > 0, mp <= m*d, n_ops >= 0", gi);
        if (p.n_ops == 0) continue;
        if (!p.U || !p.O || !p.out)
            return perr(ROT_ERR_INVALID_ARG, "group %d: null buffer", gi);
        if (p.ldu < p.mp || p.ldo < p.m || p.ldout < p.mp || (int64_t)p.d * p.ldu > INT32_MAX)
            return perr(ROT_ERR_INVALID_ARG, "group %d: leading dimensions below mp, m, mp (or d*ldu >= 2^31)", gi);
        if (p.stride_o < (int64_t)(p.m - 1) * p.ldo + p.m || p.stride_out < (int64_t)(p.mp - 1) * p.ldout + p.mp)
            return perr(ROT_ERR_INVALID_ARG, "group %d: operator stride too small", gi);
        min_ws = std::max(min_ws, ((size_t)p.m * p.d * p.ldu * 4 + 255) / 256 * 256);
    }
    if (min_ws > 0 && (!workspace || workspace_bytes < min_ws))
        return perr(ROT_ERR_WORKSPACE, "workspace %zu bytes < one operator's intermediate (%zu)", workspace_bytes, min_ws);

    rot_plan_s* P = new rot_plan_s();
    P->use_graph = !(flags & ROT_PLAN_NO_GRAPH) && !graphs_disabled();
    P->groups = rg;
    // the caller's pending work on its buffers finishes before tuning writes
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking);
    int dev = 0, n_cu = 256;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    hipDeviceProp_t props;
    if (e == hipSuccess) e = hipGetDeviceProperties(&props, dev);
    if (e != hipSuccess) {
        destroy(P);
        return perr(ROT_ERR_HIP, "plan setup: %s", hipGetErrorString(e));
    }
    std::string arch = props.gcnArchName;
    arch = arch.substr(0, arch.find(':'));

    // 1. size classes
    std::map<std::pair<int, int>, int> cls_of;
    std::vector<std::vector<int>> members;
    for (int gi = 0; gi < n_groups; gi++) {
        const rot_problem& p = rg[gi];
        if (p.n_ops == 0) continue;
        const std::pair<int, int> key{ceil_log2((int64_t)p.m * p.d), ceil_log2(p.mp)};
        auto it = cls_of.find(key);
        if (it == cls_of.end()) {
            it = cls_of.emplace(key, (int)P->classes.size()).first;
            rot_plan_s::Class c;
            char buf[128];
            snprintf(buf, sizeof buf, "%s|cu%d|fp32|md2^%d|mp2^%d", arch.c_str(), n_cu, key.first, key.second);
            c.key = buf;
            P->classes.push_back(c);
            members.emplace_back();
        }
        members[it->second].push_back(gi);
        const double f = 2.0 * p.m * p.m * p.d * p.mp + 2.0 * p.m * p.d * (double)p.mp * p.mp;
        P->classes[it->second].flops += f * p.n_ops;
        P->classes[it->second].n_ops += p.n_ops;
    }
    // largest classes first
    std::vector<int> order(P->classes.size());
    for (size_t i = 0; i < order.size(); i++) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return P->classes[a].flops > P->classes[b].flops; });

    // 2-3. chunks and work-lists
    char* ws = static_cast<char*>(workspace);
    for (int ci : order) {
        std::vector<GroupedProblem> s1, s2;
        std::vector<std::pair<int, int>> srcs;
        std::vector<const float*> ts;
        size_t used = 0;
        double chunk_flops = 0;
        auto flush = [&]() -> hipError_t {
            if (s1.empty()) return hipSuccess;
            for (int stage = 1; stage <= 2; stage++) {
                rot_plan_s::Launch L;
                L.cls = ci;
                L.stage = stage;
                L.flops = chunk_flops / 2;
                L.src = srcs;
                L.t = ts;
                const std::vector<GroupedProblem>& v = stage == 1 ? s1 : s2;
                hipError_t err = hipMalloc(&L.probs, sizeof(GroupedProblem) * v.size());
                if (err == hipSuccess)
                    err = hipMemcpy(L.probs, v.data(), sizeof(GroupedProblem) * v.size(), hipMemcpyHostToDevice);
                if (err == hipSuccess) err = hipMalloc(&L.counter, sizeof(int));
                P->launches.push_back(L);
                P->host_probs.push_back(v);
                if (err != hipSuccess) return err;
            }
            s1.clear();
            s2.clear();
            srcs.clear();
            ts.clear();
            used = 0;
            chunk_flops = 0;
            return hipSuccess;
        };
        for (int gi : members[ci]) {
            const rot_problem& p = rg[gi];
            // T_b takes U's row layout ((m*d) x ldu), so stage 1 reads U_r as
            // one matrix of row stride d*ldu over (d-1)*ldu + mp columns
            const size_t tb = ((size_t)p.m * p.d * p.ldu * 4 + 255) / 256 * 256;
            for (int b = 0; b < p.n_ops; b++) {
                if (used + tb > workspace_bytes) {
                    e = flush();
                    if (e != hipSuccess) break;
                }
                const float* T = reinterpret_cast<const float*>(ws + used);
                s1.push_back(stage_problem(p, b, T, 1));
                s2.push_back(stage_problem(p, b, T, 2));
                srcs.emplace_back(gi, b);
                ts.push_back(T);
                used += tb;
                chunk_flops += 2.0 * p.m * p.m * p.d * p.mp + 2.0 * p.m * p.d * (double)p.mp * p.mp;
            }
            if (e != hipSuccess) break;
        }
        if (e == hipSuccess) e = flush();
        if (e != hipSuccess) break;
    }
    if (e != hipSuccess) {
        destroy(P);
        return perr(ROT_ERR_HIP, "plan work-lists: %s", hipGetErrorString(e));
    }

    // 4. tile shape and schedule per class
    {
        for (int ci = 0; ci < (int)P->classes.size() && e == hipSuccess; ci++) {
            rot_plan_s::Class& c = P->classes[ci];
            GroupedShape shape;
            bool dynamic;
            int grid;
            if (!(flags & ROT_PLAN_RETUNE) && cached_choice(c.key, &shape, &dynamic, &grid) &&
                (shape != GroupedShape::k128d || class_whole(P, ci))) {
                c.shape = shape;
                c.dynamic = dynamic;
                c.grid = grid;
            } else if (!(flags & ROT_PLAN_NO_TUNE)) {
                e = tune_class(P, ci, n_cu);
                if (e == hipSuccess)
                    tune_put(c.key, {shape_name(c.shape), c.dynamic ? "dynamic" : "static", std::to_string(c.grid)});
            } else {
                c.shape = GroupedShape::k128;  // default: one workgroup per 128 x 128 tile
                c.dynamic = false;
                c.grid = 0;
            }
        }
    }
    const int sched = forced_schedule();
    for (auto& c : P->classes) {
        if (sched >= 0) {
            c.dynamic = sched == 1;
            if (c.dynamic && c.grid <= 0) c.grid = 2 * n_cu;  // the queue needs persistent workgroups
        }
        log_msg(2, "plan class %s: %d operators, tile %s, %s schedule, grid %d%s", c.key.c_str(), c.n_ops,
                shape_name(c.shape), c.dynamic ? "dynamic" : "static", c.grid, c.tuned ? " (tuned now)" : "");
    }
    for (size_t li = 0; li < P->launches.size() && e == hipSuccess; li++)
        e = upload_tiles(P->launches[li], P->host_probs[li], P->classes[P->launches[li].cls].shape);
    if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
    if (e != hipSuccess) {
        destroy(P);
        return perr(ROT_ERR_HIP, "plan tuning: %s", hipGetErrorString(e));
    }

    // 5. capture
    if (P->use_graph) {
        e = hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t e2 = issue_all(P, P->stream, false);
            e = hipStreamEndCapture(P->stream, &P->graph);
            if (e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            // graphs unavailable: fall back to direct launches
            (void)hipGetLastError();
            if (P->graph) (void)hipGraphDestroy(P->graph);
            P->graph = nullptr;
            P->exec = nullptr;
            P->use_graph = false;
            e = hipSuccess;
        }
    }
    *out = P;
    return ROT_OK;
}

rot_status rot_plan_rebind(rot_plan plan, const rot_problem* groups, int32_t n_groups, void* stream) {
    rot::TraceRange trace_("rot_plan_rebind");
    if (!plan) return perr(ROT_ERR_INVALID_ARG, "null plan");
    if (n_groups != (int32_t)plan->groups.size() || (n_groups > 0 && !groups))
        return perr(ROT_ERR_INVALID_ARG, "rebind needs the plan's %zu groups", plan->groups.size());
    std::vector<rot_problem> rg(groups, groups + n_groups);
    for (int gi = 0; gi < n_groups; gi++) {
        rot_problem& p = rg[gi];
        if (p.ldu == 0) p.ldu = p.mp;
        if (p.ldo == 0) p.ldo = p.m;
        if (p.ldout == 0) p.ldout = p.mp;
        const rot_problem& q = plan->groups[gi];
        if (p.m != q.m || p.d != q.d || p.mp != q.mp || p.n_ops != q.n_ops || p.ldu != q.ldu || p.ldo != q.ldo ||
            p.ldout != q.ldout || p.stride_o != q.stride_o || p.stride_out != q.stride_out)
            return perr(ROT_ERR_INVALID_ARG, "group %d: shape, leading dimensions or strides differ from the plan's",
                        gi);
        if (p.n_ops > 0 && (!p.U || !p.O || !p.out)) return perr(ROT_ERR_INVALID_ARG, "group %d: null buffer", gi);
    }
    size_t total = 0;
    for (auto& L : plan->launches) total += L.src.size();
    hipError_t e = hipSuccess;
    if (!plan->staging) {
        e = hipHostMalloc(reinterpret_cast<void**>(&plan->staging), sizeof(GroupedProblem) * std::max<size_t>(total, 1));
        if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->staged, hipEventDisableTiming);
        if (e != hipSuccess) return perr(ROT_ERR_HIP, "rot_plan_rebind setup: %s", hipGetErrorString(e));
        plan->staging_count = total;
    }
    // the previous rebind's copies must have left the staging buffer
    e = hipEventSynchronize(plan->staged);
    if (e != hipSuccess) return perr(ROT_ERR_HIP, "rot_plan_rebind: %s", hipGetErrorString(e));
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the new tables; a class tuned to the k128d shape needs every problem
    // whole (16-byte aligned U and O), checked before anything changes
    size_t at = 0;
    for (size_t li = 0; li < plan->launches.size(); li++) {
        auto& L = plan->launches[li];
        GroupedProblem* dst = plan->staging + at;
        const bool need_whole = plan->classes[L.cls].shape == GroupedShape::k128d;
        for (size_t k = 0; k < L.src.size(); k++) {
            dst[k] = stage_problem(rg[L.src[k].first], L.src[k].second, L.t[k], L.stage);
            if (need_whole && !(dst[k].flags & kGroupedWhole))
                return perr(ROT_ERR_INVALID_ARG,
                            "rot_plan_rebind: group %d's U or O is not 16-byte aligned, which the plan's kernels for "
                            "its size class need (the plan was created with aligned buffers)",
                            L.src[k].first);
        }
        at += L.src.size();
    }
    at = 0;
    for (size_t li = 0; li < plan->launches.size() && e == hipSuccess; li++) {
        auto& L = plan->launches[li];
        GroupedProblem* dst = plan->staging + at;
        plan->host_probs[li].assign(dst, dst + L.src.size());
        // in stream order: replays enqueued before this call read the old tables
        e = hipMemcpyAsync(L.probs, dst, sizeof(GroupedProblem) * L.src.size(), hipMemcpyHostToDevice, s);
        at += L.src.size();
    }
    if (e == hipSuccess) e = hipEventRecord(plan->staged, s);
    if (e != hipSuccess) return perr(ROT_ERR_HIP, "rot_plan_rebind: %s", hipGetErrorString(e));
    plan->groups = rg;
    return ROT_OK;
}

rot_status rot_plan_execute(rot_plan plan, void* stream) {
    rot::TraceRange trace_("rot_plan_execute");
    if (!plan) return perr(ROT_ERR_INVALID_ARG, "null plan");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = plan->use_graph ? prof_timed("plan_graph_fp32", s, [&] { return hipGraphLaunch(plan->exec, s); })
                                   : issue_all(plan, s, true);
    return e == hipSuccess ? ROT_OK : perr(ROT_ERR_HIP, "rot_plan_execute: %s", hipGetErrorString(e));
}

int32_t rot_plan_describe(rot_plan plan, char* buf, size_t len) {
    if (!plan) return -1;
    std::ostringstream os;
    os << "{\"graph\": " << (plan->use_graph ? "true" : "false") << ", \"launches\": " << plan->launches.size()
       << ", \"classes\": [";
    for (size_t i = 0; i < plan->classes.size(); i++) {
        const auto& c = plan->classes[i];
        os << (i ? ", " : "") << "{\"key\": \"" << c.key << "\", \"ops\": " << c.n_ops << ", \"gflop\": "
           << c.flops / 1e9 << ", \"tile\": " << grouped_tile_edge(c.shape)
           << ", \"lds_direct\": " << (c.shape == GroupedShape::k128d ? "true" : "false") << ", \"schedule\": \""
           << (c.dynamic ? "dynamic" : "static") << "\", \"grid\": " << c.grid << ", \"tuned_now\": "
           << (c.tuned ? "true" : "false") << "}";
    }
    os << "]}";
    const std::string s = os.str();
    if (buf && len) {
        const size_t n = std::min(len - 1, s.size());
        memcpy(buf, s.data(), n);
        buf[n] = 0;
    }
    return (int32_t)s.size();
}

rot_status rot_plan_destroy(rot_plan plan) {
    if (plan) {
        (void)hipStreamSynchronize(plan->stream);
        destroy(plan);
    }
    return ROT_OK;
}

}  // extern "C"
