// Host side of librot: argument validation, workspace carving, operator
// chunking and kernel dispatch for the C ABI declared in librot.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "rot_internal.h"

namespace rot {

hipError_t split_bf16(const float* x, int64_t n, uint16_t* hi, uint16_t* lo, hipStream_t stream);
size_t bf16_group_workspace(int m, int d, int mp, int ops);
bool bf16_shape_supported(int m, int d, int mp);
hipError_t bf16_choice(const rot_problem& p, int nb, bool symmetric, void* ws, bool may_tune, hipStream_t stream,
                       Bf16Choice* choice);
hipError_t rotate_bf16(const rot_problem& p, int b0, int nb, void* ws, bool symmetric, const Bf16Choice& choice,
                       hipStream_t stream);
bool bf16_backward_supported(int m, int d, int mp);
size_t bf16_backward_workspace(int m, int d, int mp, int ops);
hipError_t backward_bf16(const rot_problem& p, int b0, int nb, const float* dout, int64_t sd, float* dO, float* dU,
                         bool sym, void* ws, hipStream_t s);
size_t blocked_workspace_bytes(const rot_blocked_problem* p);
rot_status blocked_validate(const rot_blocked_problem* p, std::string* why);
hipError_t rotate_blocked(const rot_blocked_problem* p, void* ws, size_t ws_bytes, hipStream_t stream);
size_t density_workspace_bytes(const rot_dm_sector* sectors, int n_sectors);
hipError_t density_basis(const rot_dm_sector* sectors, int n_sec, int64_t m_keep, int32_t* kept, double* eps,
                         void* workspace, hipStream_t stream, bool* converged);

namespace {

thread_local std::string g_last_error;

rot_status fail(rot_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    log_msg(1, "%s: %s", rot_status_string(s), buf);
    return s;
}

rot_status hip_fail(hipError_t e, const char* where) {
    return fail(ROT_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;

// ---- per-kernel event timing (rot_profile_enable / rot_profile_read) ----
struct ProfRecord {
    std::string name;
    hipEvent_t start, stop;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRecord> g_prof;

template <class F>
hipError_t timed(const char* name, hipStream_t s, F&& launch) {
    bool on;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        on = g_prof_on;
    }
    if (!on) return launch();
    ProfRecord r{name, nullptr, nullptr};
    hipError_t e = hipEventCreate(&r.start);
    if (e == hipSuccess) e = hipEventCreate(&r.stop);
    if (e == hipSuccess) e = hipEventRecord(r.start, s);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(r.stop, s);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.push_back(r);
    return hipSuccess;
}

void prof_clear_locked() {
    for (auto& r : g_prof) {
        if (r.start) (void)hipEventDestroy(r.start);
        if (r.stop) (void)hipEventDestroy(r.stop);
    }
    g_prof.clear();
}

inline size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

size_t elem_size(rot_precision p) { return p == ROT_FP64 ? 8 : 4; }

bool valid_precision(int p) { return p == ROT_FP64 || p == ROT_FP32 || p == ROT_SPLIT_BF16; }

// A group with its leading dimensions resolved (0 selects the packed value).
rot_problem resolved(const rot_problem& p) {
    rot_problem q = p;
    if (q.ldu == 0) q.ldu = q.mp;
    if (q.ldo == 0) q.ldo = q.m;
    if (q.ldout == 0) q.ldout = q.mp;
    return q;
}

std::vector<rot_problem> resolved_all(const rot_problem* groups, int n) {
    std::vector<rot_problem> v(groups, groups + std::max(n, 0));
    for (auto& q : v) q = resolved(q);
    return v;
}

// Bytes of one operator's stage-1 intermediate T_b ((m*d) x mp, row stride
// ldu: T_b takes U's row layout so stage 1 can read U_r with one leading
// dimension, see stage1()).
size_t t_bytes(const rot_problem& p, rot_precision prec) {
    return align_up((size_t)p.m * p.d * p.ldu * elem_size(prec));
}

// Bytes of U packed to row stride mp (the adjoint's products read U_r, the
// m x d*mp view, which only a packed U provides).
size_t packed_u_bytes(const rot_problem& p, rot_precision prec) {
    return p.ldu == p.mp ? 0 : align_up((size_t)p.m * p.d * p.mp * elem_size(prec));
}

// Stage 2 split over K for small outputs: when the chunk's stage-2 output
// has fewer than 256 tiles of 128 x 128 (too few workgroups to fill the chip)
// and K = m*d is long, K is cut into parts of kp (a multiple of 16, at least
// 64) computed by separate workgroups into partial sums that are added in a
// fixed order.  Returns the number of parts (1: no split) for `ops` operators.
int stage2_parts(const rot_problem& p, int ops, int* kp) {
    const int64_t t = (p.mp + kGemmTile - 1) / kGemmTile;
    const int64_t tiles = t * t * ops;
    const int64_t K = (int64_t)p.m * p.d;
    *kp = (int)K;
    if (tiles >= 256 || K < 128) return 1;
    int64_t parts = std::min<int64_t>({8, (512 + tiles - 1) / tiles, K / 64});
    if (parts < 2) return 1;
    const int64_t k = ((K + parts - 1) / parts + 15) / 16 * 16;
    *kp = (int)k;
    return (int)((K + k - 1) / k);
}

// Bytes of one operator's partial stage-2 sums when split into `parts`.
size_t stage2_part_bytes(const rot_problem& p, int parts, size_t es) {
    return parts > 1 ? (size_t)parts * p.mp * p.mp * es : 0;
}

// The dU reduction of rot_backward is one GEMM with M = m, N = d*mp and a K
// range over every operator of a chunk; when its 128x128 output tiles are too
// few to fill the chip the operator range is split into parts, each reduced
// into its own partial dU (one workspace slot of t_bytes), and the parts are
// summed in fixed order.  Returns the number of parts (0: no split) for a
// chunk of `ops` operators.
int du_split_parts(const rot_problem& p, int ops) {
    const int64_t tiles = (((int64_t)p.m + kGemmTile - 1) / kGemmTile) *
                          (((int64_t)p.d * p.mp + kGemmTile - 1) / kGemmTile);
    int parts = (int)std::min<int64_t>(8, (4 * 256 + tiles - 1) / tiles);
    parts = std::min(parts, ops);
    return parts > 1 ? parts : 0;
}

// p must be resolved (leading dimensions filled in).
rot_status validate_group(const rot_problem& p, int gi) {
    if (p.m <= 0 || p.d <= 0 || p.mp <= 0)
        return fail(ROT_ERR_INVALID_ARG, "group %d: m, d, mp must be positive (m=%d d=%d mp=%d)", gi,
                    p.m, p.d, p.mp);
    const int64_t md = (int64_t)p.m * p.d, dmp = (int64_t)p.d * p.mp;
    if (md > INT32_MAX || dmp > INT32_MAX)
        return fail(ROT_ERR_INVALID_ARG, "group %d: m*d or d*mp exceeds 2^31-1", gi);
    if (p.mp > md) return fail(ROT_ERR_INVALID_ARG, "group %d: mp=%d exceeds m*d=%lld", gi, p.mp, (long long)md);
    if (p.n_ops < 0) return fail(ROT_ERR_INVALID_ARG, "group %d: negative n_ops", gi);
    if (p.n_ops == 0) return ROT_OK;
    if (!p.U || !p.O || !p.out) return fail(ROT_ERR_INVALID_ARG, "group %d: null U, O or out", gi);
    if (p.ldu < p.mp || p.ldo < p.m || p.ldout < p.mp)
        return fail(ROT_ERR_INVALID_ARG, "group %d: leading dimensions ldu=%lld ldo=%lld ldout=%lld below mp, m, mp",
                    gi, (long long)p.ldu, (long long)p.ldo, (long long)p.ldout);
    if (p.ldu > INT32_MAX || (int64_t)p.d * p.ldu > INT32_MAX)
        return fail(ROT_ERR_INVALID_ARG, "group %d: d*ldu exceeds 2^31-1", gi);
    if (p.stride_o < (int64_t)(p.m - 1) * p.ldo + p.m)
        return fail(ROT_ERR_INVALID_ARG, "group %d: stride_o %lld < (m-1)*ldo + m", gi, (long long)p.stride_o);
    if (p.stride_out < (int64_t)(p.mp - 1) * p.ldout + p.mp)
        return fail(ROT_ERR_INVALID_ARG, "group %d: stride_out %lld < (mp-1)*ldout + mp", gi,
                    (long long)p.stride_out);
    return ROT_OK;
}

bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + nb && pb < pa + na;
}

rot_status validate_outputs_disjoint(const rot_problem& p, rot_precision prec, int gi) {
    const size_t es = elem_size(prec);
    const size_t n_out = ((size_t)(p.n_ops - 1) * p.stride_out + (size_t)(p.mp - 1) * p.ldout + p.mp) * es;
    const size_t n_o = ((size_t)(p.n_ops - 1) * p.stride_o + (size_t)(p.m - 1) * p.ldo + p.m) * es;
    const size_t n_u = ((size_t)p.m * p.d - 1) * p.ldu * es + (size_t)p.mp * es;
    if (ranges_overlap(p.out, n_out, p.O, n_o) || ranges_overlap(p.out, n_out, p.U, n_u))
        return fail(ROT_ERR_INVALID_ARG, "group %d: out overlaps U or O", gi);
    return ROT_OK;
}

// Stage 1: T_b = O_b * U_r for nb operators from b0.  With row stride ldu,
// U_r(j, c) = U[j*d*ldu + c] for c = s*ldu + beta is one matrix of row stride
// d*ldu; its columns beta >= mp of s < d-1 are U's row padding, so the
// product spans N = (d-1)*ldu + mp columns and T_b gets U's row layout
// ((m*d) x ldu, batch stride m*d*ldu).  Padding columns of T_b hold products
// with U's padding and are never read.
GemmDesc stage1(const rot_problem& p, int b0, int nb, void* T, size_t es) {
    GemmDesc g{};
    g.M = p.m;
    g.N = (int)((int64_t)(p.d - 1) * p.ldu + p.mp);
    g.K = p.m;
    g.batch = nb;
    g.kbatch = 1;
    g.A = static_cast<const char*>(p.O) + (size_t)b0 * p.stride_o * es;
    g.lda = p.ldo;
    g.a_bs = p.stride_o;
    g.a_kcontig = true;  // O_b(i, j) at O_b[i*ldo + j]
    g.B = p.U;
    g.ldb = (int64_t)p.d * p.ldu;
    g.b_bs = 0;
    g.b_kcontig = false;  // U_r(j, c) at U[j*d*ldu + c]
    g.C = T;
    g.ldc = (int64_t)p.d * p.ldu;
    g.c_bs = (int64_t)p.m * p.d * p.ldu;
    return g;
}

// Stage 2: out_b = U^T * T_b, T_b viewed as (m*d) x mp with row stride ldu.
GemmDesc stage2(const rot_problem& p, int b0, int nb, const void* T, size_t es) {
    GemmDesc g{};
    g.M = p.mp;
    g.N = p.mp;
    g.K = p.m * p.d;
    g.batch = nb;
    g.kbatch = 1;
    g.A = p.U;
    g.lda = p.ldu;
    g.a_bs = 0;
    g.a_kcontig = false;  // A(alpha, r) = U[r*ldu + alpha]
    g.B = T;
    g.ldb = p.ldu;
    g.b_bs = (int64_t)p.m * p.d * p.ldu;
    g.b_kcontig = false;  // T_b(r, beta) at T_b[r*ldu + beta]
    g.C = static_cast<char*>(p.out) + (size_t)b0 * p.stride_out * es;
    g.ldc = p.ldout;
    g.c_bs = p.stride_out;
    return g;
}

hipError_t gemm(rot_precision prec, const GemmDesc& g, hipStream_t s, const char* what) {
    const bool f64 = prec == ROT_FP64;
    std::string name = std::string(what) + (f64 ? "_fp64" : "_fp32");
    return timed(name.c_str(), s, [&] { return f64 ? gemm_f64(g, s) : gemm_f32(g, s); });
}

// Split-K for a single GEMM whose output has too few 128 x 128 tiles to fill
// the chip: K is cut into `parts` equal ranges (the remainder joins part 0),
// each part's product goes to its own partial sum (parts x M x N), and the
// partials are added in fixed order.  Returns the number of parts (1: no
// split) for an output of M x N over K.
int split_k_parts(int M, int N, int64_t K) {
    const int64_t tiles = (((int64_t)M + kGemmTile - 1) / kGemmTile) * (((int64_t)N + kGemmTile - 1) / kGemmTile);
    int64_t parts = (1024 + tiles - 1) / tiles;
    parts = std::min<int64_t>(parts, 256);
    parts = std::min<int64_t>(parts, std::max<int64_t>(1, K / 256));
    return (int)std::max<int64_t>(1, parts);
}

size_t split_k_scratch(int M, int N, int64_t K, size_t es) {
    const int parts = split_k_parts(M, N, K);
    return parts > 1 ? align_up((size_t)parts * M * N * es) : 0;
}

// C = A B (batch = kbatch = 1, no accumulation) through `scratch` of at least
// split_k_scratch(M, N, K, es) bytes; plain GEMM when no split pays.
hipError_t gemm_split_k(rot_precision prec, const GemmDesc& g, void* scratch, hipStream_t s, const char* what) {
    const int parts = split_k_parts(g.M, g.N, g.K);
    if (parts <= 1) return gemm(prec, g, s, what);
    const size_t es = elem_size(prec);
    const int kp = g.K / parts, rem = g.K % parts;
    GemmDesc p = g;
    p.K = kp;
    p.batch = parts;
    p.a_bs = g.a_kcontig ? kp : (int64_t)kp * g.lda;  // next K range of A
    p.b_bs = g.b_kcontig ? kp : (int64_t)kp * g.ldb;
    p.C = scratch;
    p.ldc = g.N;
    p.c_bs = (int64_t)g.M * g.N;
    p.accumulate = false;
    hipError_t e = gemm(prec, p, s, what);
    if (e == hipSuccess && rem > 0) {
        GemmDesc t = p;
        t.batch = 1;
        t.K = rem;
        t.A = static_cast<const char*>(g.A) + (size_t)parts * p.a_bs * es;
        t.B = static_cast<const char*>(g.B) + (size_t)parts * p.b_bs * es;
        t.accumulate = true;
        e = gemm(prec, t, s, what);
    }
    if (e != hipSuccess) return e;
    if (g.ldc == g.N)
        return timed("split_k_sum", s, [&] {
            return sum_parts(g.C, scratch, (int64_t)g.M * g.N, parts, (int64_t)g.M * g.N, false, prec == ROT_FP64, s);
        });
    // strided C: add the parts row by row
    return timed("split_k_sum", s, [&] {
        hipError_t err = hipSuccess;
        for (int r = 0; r < g.M && err == hipSuccess; r++)
            err = sum_parts(static_cast<char*>(g.C) + (size_t)r * g.ldc * es,
                            static_cast<char*>(scratch) + (size_t)r * g.N * es, g.N, parts, (int64_t)g.M * g.N,
                            false, prec == ROT_FP64, s);
        return err;
    });
}

}  // namespace

rot_status set_error(rot_status s, const char* msg) {
    g_last_error = msg;
    log_msg(1, "%s: %s", rot_status_string(s), msg);
    return s;
}

hipError_t prof_timed(const char* name, hipStream_t stream, const std::function<hipError_t()>& launch) {
    return timed(name, stream, launch);
}

}  // namespace rot

using namespace rot;

extern "C" {

const char* rot_status_string(rot_status s) {
    switch (s) {
        case ROT_OK: return "ROT_OK";
        case ROT_ERR_INVALID_ARG: return "ROT_ERR_INVALID_ARG";
        case ROT_ERR_UNSUPPORTED: return "ROT_ERR_UNSUPPORTED";
        case ROT_ERR_WORKSPACE: return "ROT_ERR_WORKSPACE";
        case ROT_ERR_HIP: return "ROT_ERR_HIP";
        case ROT_ERR_NOT_ISOMETRY: return "ROT_ERR_NOT_ISOMETRY";
        case ROT_ERR_NOT_CONVERGED: return "ROT_ERR_NOT_CONVERGED";
    }
    return "unknown rot_status";
}

const char* rot_last_error(void) { return g_last_error.c_str(); }

rot_status rot_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (on) prof_clear_locked();
    g_prof_on = on != 0;
    return ROT_OK;
}

int32_t rot_profile_read(char* buf, size_t len) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    std::map<std::string, std::pair<int, double>> agg;
    int32_t rc = 0;
    for (auto& r : g_prof) {
        float ms = 0.f;
        if (hipEventSynchronize(r.stop) != hipSuccess || hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) {
            rc = -1;
            continue;
        }
        auto& a = agg[r.name];
        a.first += 1;
        a.second += ms;
    }
    prof_clear_locked();
    std::string out;
    char line[256];
    for (auto& kv : agg) {
        snprintf(line, sizeof(line), "%s %d %.6f\n", kv.first.c_str(), kv.second.first, kv.second.second);
        out += line;
    }
    if (buf && len) {
        const size_t n = std::min(len - 1, out.size());
        memcpy(buf, out.data(), n);
        buf[n] = 0;
    }
    return rc < 0 ? rc : (int32_t)agg.size();
}

int32_t rot_version(void) { return 100; }

size_t rot_workspace_size(const rot_problem* groups, int32_t n_groups, rot_precision prec,
                          int32_t ops_per_chunk, int32_t for_backward) {
    if (n_groups < 0 || (n_groups > 0 && !groups) || !valid_precision(prec)) return 0;
    size_t need = 0;
    for (int gi = 0; gi < n_groups; gi++) {
        const rot_problem p = resolved(groups[gi]);
        if (validate_group(p, gi) != ROT_OK) return 0;
        if (p.n_ops == 0) continue;
        const int ops = ops_per_chunk > 0 ? std::min(ops_per_chunk, p.n_ops) : p.n_ops;
        const rot_precision tp = prec == ROT_FP64 ? ROT_FP64 : ROT_FP32;
        size_t g;
        if (prec == ROT_SPLIT_BF16 && !for_backward) {
            g = bf16_group_workspace(p.m, p.d, p.mp, ops);
        } else if (prec == ROT_SPLIT_BF16) {
            g = packed_u_bytes(p, tp) + bf16_backward_workspace(p.m, p.d, p.mp, ops);
        } else if (for_backward) {
            rot_problem packed = p;
            packed.ldu = p.mp;  // the adjoint works on U packed to row stride mp
            g = packed_u_bytes(p, tp) + (size_t)(ops + du_split_parts(p, ops)) * t_bytes(packed, tp);
        } else {
            // with more than one operator per chunk, room for the split stage-2 partial sums
            int kp = 0;
            const int parts = ops > 1 || ops_per_chunk <= 0 ? stage2_parts(p, ops, &kp) : 1;
            g = (size_t)ops * t_bytes(p, tp) + align_up((size_t)ops * stage2_part_bytes(p, parts, elem_size(tp)));
        }
        need = std::max(need, g);
    }
    return need;
}

rot_status rot_batch(const rot_problem* groups, int32_t n_groups, rot_precision prec, void* workspace,
                     size_t workspace_bytes, void* stream) {
    return rot_batch_ex(groups, n_groups, prec, 0u, workspace, workspace_bytes, stream);
}

rot_status rot_batch_ex(const rot_problem* groups, int32_t n_groups, rot_precision prec, uint32_t flags,
                        void* workspace, size_t workspace_bytes, void* stream) {
    rot::TraceRange trace_("rot_batch_ex");
    if (n_groups < 0 || (n_groups > 0 && !groups))
        return fail(ROT_ERR_INVALID_ARG, "groups is null or n_groups negative");
    if (!valid_precision(prec)) return fail(ROT_ERR_INVALID_ARG, "unknown precision %d", (int)prec);
    if (flags & ~ROT_ASSUME_SYMMETRIC_O) return fail(ROT_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    const bool sym = flags & ROT_ASSUME_SYMMETRIC_O;
    const std::vector<rot_problem> rg = resolved_all(groups, n_groups);
    for (int gi = 0; gi < n_groups; gi++) {
        rot_status s = validate_group(rg[gi], gi);
        if (s != ROT_OK) return s;
        if (rg[gi].n_ops > 0) {
            s = validate_outputs_disjoint(rg[gi], prec, gi);
            if (s != ROT_OK) return s;
            if (prec == ROT_SPLIT_BF16 && !bf16_shape_supported(groups[gi].m, groups[gi].d, groups[gi].mp))
                return fail(ROT_ERR_UNSUPPORTED,
                            "group %d: split-bf16 operand arrays must stay below 2 GiB (m=%d d=%d mp=%d); use ROT_FP32",
                            gi, groups[gi].m, groups[gi].d, groups[gi].mp);
        }
    }
    const size_t min_ws = rot_workspace_size(groups, n_groups, prec, 1, 0);
    if (min_ws > 0) {
        if (!workspace) return fail(ROT_ERR_WORKSPACE, "workspace is null (need %zu bytes)", min_ws);
        if (workspace_bytes < min_ws)
            return fail(ROT_ERR_WORKSPACE, "workspace %zu bytes < minimum %zu", workspace_bytes, min_ws);
        if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
            return fail(ROT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t es = elem_size(prec);
    for (int gi = 0; gi < n_groups; gi++) {
        const rot_problem& p = rg[gi];
        if (p.n_ops == 0) continue;
        if (prec == ROT_SPLIT_BF16) {
            int chunk = 1;
            while (chunk < p.n_ops && bf16_group_workspace(p.m, p.d, p.mp, chunk + 1) <= workspace_bytes)
                chunk++;
            // tile configuration per stage: cached, or timed on this shape's first
            // call (never while the stream is being captured)
            hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
            const bool capturing = hipStreamIsCapturing(s, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone;
            Bf16Choice choice;
            hipError_t e = bf16_choice(p, chunk, sym, workspace, !capturing, s, &choice);
            if (e != hipSuccess) return hip_fail(e, "rot_batch split-bf16 tuning");
            for (int b0 = 0; b0 < p.n_ops; b0 += chunk) {
                const int nb = std::min(chunk, p.n_ops - b0);
                e = rotate_bf16(p, b0, nb, workspace, sym, choice, s);
                if (e != hipSuccess) return hip_fail(e, "rot_batch split-bf16");
            }
            continue;
        }
        if (prec == ROT_FP64 && !sym && rotate_small_f64_applies(p)) {
            // small blocks: both stages in one launch, no intermediate
            hipError_t e = timed("small_fp64", s, [&] { return rotate_small_f64(p, s); });
            if (e != hipSuccess) return hip_fail(e, "rot_batch small fp64");
            continue;
        }
        const size_t per_op = t_bytes(p, prec);
        // split-K stage 2 (general output only) when the workspace holds the
        // whole batch with its partial sums
        int kp = 0;
        int parts = sym ? 1 : stage2_parts(p, p.n_ops, &kp);
        const size_t need_split = (size_t)p.n_ops * per_op + align_up((size_t)p.n_ops * stage2_part_bytes(p, parts, es));
        if (parts > 1 && workspace_bytes < need_split) parts = 1;
        const int chunk = parts > 1 ? p.n_ops : (int)std::min<size_t>((size_t)p.n_ops, workspace_bytes / per_op);
        for (int b0 = 0; b0 < p.n_ops; b0 += chunk) {
            const int nb = std::min(chunk, p.n_ops - b0);
            hipError_t e = gemm(prec, stage1(p, b0, nb, workspace, es), s, "stage1");
            if (e == hipSuccess && parts > 1) {
                // parts x nb packed mp x mp partial products after the intermediates
                char* partial = static_cast<char*>(workspace) + (size_t)nb * per_op;
                GemmDesc g2 = stage2(p, b0, nb, workspace, es);
                g2.C = partial;
                g2.ldc = p.mp;
                g2.c_bs = (int64_t)p.mp * p.mp;
                g2.parts = parts;
                g2.kp = kp;
                g2.c_ps = (int64_t)nb * p.mp * p.mp;
                e = gemm(prec, g2, s, "stage2");
                if (e == hipSuccess)
                    e = timed("stage2_sum", s, [&] {
                        return sum_parts_2d(static_cast<char*>(p.out) + (size_t)b0 * p.stride_out * es, p.ldout,
                                            p.stride_out, partial, p.mp, p.mp, nb, parts, g2.c_ps, prec == ROT_FP64, s);
                    });
            } else if (e == hipSuccess) {
                GemmDesc g2 = stage2(p, b0, nb, workspace, es);
                g2.upper = sym;
                e = gemm(prec, g2, s, sym ? "stage2sym" : "stage2");
            }
            if (e != hipSuccess) return hip_fail(e, "rot_batch launch");
        }
    }
    return ROT_OK;
}

namespace {

rot_status validate_site(const rot_site_problem& p, rot_precision prec, int gi) {
    if (p.m <= 0 || p.d <= 0 || p.mp <= 0 || p.n_ops < 0)
        return fail(ROT_ERR_INVALID_ARG, "site group %d: m, d, mp must be positive and n_ops >= 0", gi);
    if (p.d > kMaxSite) return fail(ROT_ERR_UNSUPPORTED, "site group %d: d = %d exceeds %d", gi, p.d, kMaxSite);
    const int64_t md = (int64_t)p.m * p.d;
    if (md > INT32_MAX || (int64_t)p.d * p.mp > INT32_MAX || p.mp > md)
        return fail(ROT_ERR_INVALID_ARG, "site group %d: need mp <= m*d and extents below 2^31", gi);
    if (p.block_kind != ROT_BLOCK_IDENTITY && p.block_kind != ROT_BLOCK_DIAGONAL && p.block_kind != ROT_BLOCK_DENSE)
        return fail(ROT_ERR_INVALID_ARG, "site group %d: unknown block_kind %d", gi, p.block_kind);
    if (p.n_ops == 0) return ROT_OK;
    if (!p.U || !p.site || !p.out) return fail(ROT_ERR_INVALID_ARG, "site group %d: null U, site or out", gi);
    if (p.block_kind == ROT_BLOCK_IDENTITY && p.X)
        return fail(ROT_ERR_INVALID_ARG, "site group %d: X must be NULL for ROT_BLOCK_IDENTITY", gi);
    if (p.block_kind != ROT_BLOCK_IDENTITY && !p.X) return fail(ROT_ERR_INVALID_ARG, "site group %d: null X", gi);
    if (p.block_kind != ROT_BLOCK_DENSE && p.n_ops != 1)
        return fail(ROT_ERR_INVALID_ARG, "site group %d: identity and diagonal kinds take n_ops = 1", gi);
    if (p.block_kind == ROT_BLOCK_DENSE && p.stride_x < (int64_t)p.m * p.m)
        return fail(ROT_ERR_INVALID_ARG, "site group %d: stride_x must be >= m*m", gi);
    if (p.stride_out < (int64_t)p.mp * p.mp)
        return fail(ROT_ERR_INVALID_ARG, "site group %d: stride_out must be >= mp*mp", gi);
    const size_t es = elem_size(prec);
    const size_t n_out = ((size_t)(p.n_ops - 1) * p.stride_out + (size_t)p.mp * p.mp) * es;
    const size_t n_u = (size_t)md * p.mp * es;
    size_t n_x = 0;
    if (p.block_kind == ROT_BLOCK_DENSE) n_x = ((size_t)(p.n_ops - 1) * p.stride_x + (size_t)p.m * p.m) * es;
    if (p.block_kind == ROT_BLOCK_DIAGONAL) n_x = (size_t)p.m * es;
    if (ranges_overlap(p.out, n_out, p.U, n_u) || (n_x && ranges_overlap(p.out, n_out, p.X, n_x)))
        return fail(ROT_ERR_INVALID_ARG, "site group %d: out overlaps U or X", gi);
    return ROT_OK;
}

// Bytes of the mixed operand U' of one group, and of one operator's T.
size_t site_up_bytes(const rot_site_problem& p, rot_precision prec) {
    return align_up((size_t)p.m * p.d * p.mp * elem_size(prec));
}

}  // namespace

size_t rot_site_workspace_size(const rot_site_problem* groups, int32_t n_groups, rot_precision prec,
                               int32_t ops_per_chunk) {
    if (n_groups < 0 || (n_groups > 0 && !groups) || (prec != ROT_FP32 && prec != ROT_FP64)) return 0;
    size_t need = 0;
    for (int gi = 0; gi < n_groups; gi++) {
        const rot_site_problem& p = groups[gi];
        if (validate_site(p, prec, gi) != ROT_OK) return 0;
        if (p.n_ops == 0) continue;
        const size_t slot = site_up_bytes(p, prec);
        if (p.block_kind != ROT_BLOCK_DENSE) {
            need = std::max(need, slot + split_k_scratch(p.mp, p.mp, (int64_t)p.m * p.d, elem_size(prec)));
            continue;
        }
        const int ops = ops_per_chunk > 0 ? std::min(ops_per_chunk, p.n_ops) : p.n_ops;
        need = std::max(need, slot * (size_t)(1 + ops));
    }
    return need;
}

rot_status rot_batch_site(const rot_site_problem* groups, int32_t n_groups, rot_precision prec, void* workspace,
                          size_t workspace_bytes, void* stream) {
    rot::TraceRange trace_("rot_batch_site");
    if (n_groups < 0 || (n_groups > 0 && !groups))
        return fail(ROT_ERR_INVALID_ARG, "null groups or negative n_groups");
    if (prec != ROT_FP32 && prec != ROT_FP64)
        return fail(prec == ROT_SPLIT_BF16 ? ROT_ERR_UNSUPPORTED : ROT_ERR_INVALID_ARG,
                    "rot_batch_site supports ROT_FP64 and ROT_FP32");
    for (int gi = 0; gi < n_groups; gi++) {
        rot_status st = validate_site(groups[gi], prec, gi);
        if (st != ROT_OK) return st;
    }
    const size_t min_ws = rot_site_workspace_size(groups, n_groups, prec, 1);
    if (min_ws > 0) {
        if (!workspace || workspace_bytes < min_ws)
            return fail(ROT_ERR_WORKSPACE, "workspace %zu bytes < minimum %zu", workspace_bytes, min_ws);
        if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
            return fail(ROT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t es = elem_size(prec);
    for (int gi = 0; gi < n_groups; gi++) {
        const rot_site_problem& sp = groups[gi];
        if (sp.n_ops == 0) continue;
        SiteMatrix S{};
        for (int k = 0; k < sp.d * sp.d; k++) S.v[k] = sp.site[k];
        char* up = static_cast<char*>(workspace);
        const void* x = sp.block_kind == ROT_BLOCK_DIAGONAL ? sp.X : nullptr;
        hipError_t e = prof_timed("site_mix", s, [&] {
            return site_mix(sp.U, sp.m, sp.d, sp.mp, S, x, up, prec == ROT_FP64, s);
        });
        if (e != hipSuccess) return hip_fail(e, "rot_batch_site mix");
        // the same shapes as a dense group: X_b in place of O_b
        rot_problem p{};
        p.m = sp.m;
        p.d = sp.d;
        p.mp = sp.mp;
        p.n_ops = sp.n_ops;
        p.U = sp.U;
        p.O = sp.X;
        p.stride_o = sp.stride_x;
        p.out = sp.out;
        p.stride_out = sp.stride_out;
        p = resolved(p);  // packed U, X and out
        if (sp.block_kind != ROT_BLOCK_DENSE) {
            // out = U'^T U: stage 2 with U' as A and U itself as B (split over K
            // when its mp x mp output has few tiles)
            GemmDesc g = stage2(p, 0, 1, sp.U, es);
            g.A = up;
            g.ldc = sp.mp;
            e = gemm_split_k(prec, g, up + site_up_bytes(sp, prec), s, "site_stage2");
            if (e != hipSuccess) return hip_fail(e, "rot_batch_site launch");
            continue;
        }
        const size_t slot = site_up_bytes(sp, prec);
        char* T = up + slot;
        const int chunk = (int)std::min<size_t>((size_t)sp.n_ops, workspace_bytes / slot - 1);
        for (int b0 = 0; b0 < sp.n_ops; b0 += chunk) {
            const int nb = std::min(chunk, sp.n_ops - b0);
            e = gemm(prec, stage1(p, b0, nb, T, es), s, "site_stage1");
            if (e == hipSuccess) {
                GemmDesc g = stage2(p, b0, nb, T, es);
                g.A = up;
                e = gemm(prec, g, s, "site_stage2");
            }
            if (e != hipSuccess) return hip_fail(e, "rot_batch_site launch");
        }
    }
    return ROT_OK;
}

size_t rot_expect_block_workspace_size(int32_t m, int32_t d, int64_t ncols, int32_t n_ops) {
    if (m <= 0 || d <= 0 || ncols <= 0 || n_ops < 0) return 0;
    return align_up((size_t)m * m * sizeof(double)) + align_up(expect_dot_scratch(n_ops)) +
           split_k_scratch(m, m, (int64_t)d * ncols, sizeof(double));
}

rot_status rot_expect_block(const double* psi, int32_t m, int32_t d, int64_t ncols, const void* Z, int32_t n_ops,
                            int64_t stride_z, rot_precision prec, double* e, void* workspace, size_t workspace_bytes,
                            void* stream) {
    rot::TraceRange trace_("rot_expect_block");
    if (m <= 0 || d <= 0 || ncols <= 0 || n_ops < 0)
        return fail(ROT_ERR_INVALID_ARG, "m, d, ncols must be positive and n_ops >= 0");
    if (prec != ROT_FP64 && prec != ROT_FP32) return fail(ROT_ERR_INVALID_ARG, "Z must be FP64 or FP32");
    if ((int64_t)d * ncols > INT32_MAX || (int64_t)m * m > INT32_MAX)
        return fail(ROT_ERR_INVALID_ARG, "extents too large");
    if (n_ops == 0) return ROT_OK;
    if (!psi || !Z || !e) return fail(ROT_ERR_INVALID_ARG, "null psi, Z or e");
    if (stride_z < (int64_t)m * m) return fail(ROT_ERR_INVALID_ARG, "stride_z must be >= m*m");
    const size_t need = rot_expect_block_workspace_size(m, d, ncols, n_ops);
    if (!workspace || workspace_bytes < need)
        return fail(ROT_ERR_WORKSPACE, "workspace %zu bytes < %zu", workspace_bytes, need);
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(ROT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* rho = static_cast<double*>(workspace);
    double* partial = reinterpret_cast<double*>(static_cast<char*>(workspace) + align_up((size_t)m * m * 8));
    char* split = static_cast<char*>(workspace) + align_up((size_t)m * m * 8) + align_up(expect_dot_scratch(n_ops));
    // rho_B[i][i'] = sum over (s, column) of psi[i*d+s][.] psi[i'*d+s][.]: psi viewed as m x (d*ncols)
    GemmDesc g{};
    g.M = m; g.N = m; g.K = (int)(d * ncols); g.batch = 1; g.kbatch = 1;
    g.A = psi; g.lda = d * ncols; g.a_kcontig = true;
    g.B = psi; g.ldb = d * ncols; g.b_kcontig = true;
    g.C = rho; g.ldc = m;
    hipError_t err = gemm_split_k(ROT_FP64, g, split, s, "expect_rho");
    if (err == hipSuccess)
        err = prof_timed("expect_dots", s, [&] {
            return expect_dots(Z, prec == ROT_FP64, stride_z, (int64_t)m * m, n_ops, rho, partial, e, s);
        });
    return err == hipSuccess ? ROT_OK : hip_fail(err, "rot_expect_block");
}

size_t rot_expect_cross_workspace_size(int32_t m, int32_t d, int32_t mR, int32_t dR, int32_t n_left,
                                       int32_t n_right, int32_t ops_per_chunk) {
    if (m <= 0 || d <= 0 || mR <= 0 || dR <= 0 || n_left < 0 || n_right < 0) return 0;
    const size_t md = (size_t)m * d, mp = (size_t)dR * mR;
    const int ops = ops_per_chunk > 0 ? std::min(ops_per_chunk, std::max(n_left, 1)) : std::max(n_left, 1);
    const size_t per_op = align_up(md * mp * 8) + align_up(mp * mp * 8);
    const size_t split = split_k_scratch(std::max(n_left, 1), std::max(n_right, 1), (int64_t)mR * mR, 8);
    return align_up((size_t)n_left * mR * mR * 8) + split + (size_t)ops * per_op;
}

rot_status rot_expect_cross(const double* psi, int32_t m, int32_t d, int32_t mR, int32_t dR, const double* Z,
                            int32_t n_left, int64_t stride_z, const double* W, int32_t n_right, int64_t stride_w,
                            double* c, void* workspace, size_t workspace_bytes, void* stream) {
    rot::TraceRange trace_("rot_expect_cross");
    if (m <= 0 || d <= 0 || mR <= 0 || dR <= 0 || n_left < 0 || n_right < 0)
        return fail(ROT_ERR_INVALID_ARG, "m, d, mR, dR must be positive, operator counts >= 0");
    const int64_t md = (int64_t)m * d, mp = (int64_t)dR * mR;
    if (md > INT32_MAX || (int64_t)m * mp > INT32_MAX || (int64_t)mR * mR > INT32_MAX)
        return fail(ROT_ERR_INVALID_ARG, "extents too large");
    if (n_left == 0 || n_right == 0) return ROT_OK;
    if (!psi || !Z || !W || !c) return fail(ROT_ERR_INVALID_ARG, "null psi, Z, W or c");
    if (stride_z < (int64_t)m * m || stride_w < (int64_t)mR * mR)
        return fail(ROT_ERR_INVALID_ARG, "stride_z must be >= m*m and stride_w >= mR*mR");
    const size_t need = rot_expect_cross_workspace_size(m, d, mR, dR, n_left, n_right, 1);
    if (!workspace || workspace_bytes < need)
        return fail(ROT_ERR_WORKSPACE, "workspace %zu bytes < minimum %zu", workspace_bytes, need);
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(ROT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(workspace);
    double* q = reinterpret_cast<double*>(base);
    const size_t q_bytes = align_up((size_t)n_left * mR * mR * 8);
    char* split = base + q_bytes;
    const size_t split_bytes = split_k_scratch(n_left, n_right, (int64_t)mR * mR, 8);
    const size_t t_bytes_op = align_up((size_t)md * mp * 8), qq_bytes_op = align_up((size_t)mp * mp * 8);
    const int chunk = (int)std::min<size_t>((size_t)n_left,
                                            (workspace_bytes - q_bytes - split_bytes) / (t_bytes_op + qq_bytes_op));
    char* T = base + q_bytes + split_bytes;
    char* Q = T + (size_t)chunk * t_bytes_op;
    hipError_t err = hipSuccess;
    for (int b0 = 0; b0 < n_left && err == hipSuccess; b0 += chunk) {
        const int nb = std::min(chunk, n_left - b0);
        // Q_b = psi^T (Z_b (x) I_d) psi: the rotation with psi in place of U (m' = dR*mR)
        rot_problem p{};
        p.m = m; p.d = d; p.mp = (int32_t)mp; p.n_ops = nb;
        p.U = psi; p.O = Z + (size_t)b0 * stride_z; p.stride_o = stride_z;
        p.out = Q; p.stride_out = mp * mp;
        p = resolved(p);  // packed psi, Z and Q
        GemmDesc g1 = stage1(p, 0, nb, T, 8);
        g1.c_bs = (int64_t)(t_bytes_op / 8);
        err = gemm(ROT_FP64, g1, s, "expect_stage1");
        if (err == hipSuccess) {
            GemmDesc g2 = stage2(p, 0, nb, T, 8);
            g2.b_bs = (int64_t)(t_bytes_op / 8);
            g2.c_bs = (int64_t)(qq_bytes_op / 8);
            err = gemm(ROT_FP64, g2, s, "expect_stage2");
        }
        if (err == hipSuccess) {
            err = prof_timed("expect_trace", s, [&] {
                return partial_trace(reinterpret_cast<const double*>(Q), (int64_t)(qq_bytes_op / 8), mR, dR, nb,
                                     q + (size_t)b0 * mR * mR, s);
            });
        }
    }
    if (err == hipSuccess) {
        // c[b][k] = sum_e q_b[e] W_k[e]
        GemmDesc g{};
        g.M = n_left; g.N = n_right; g.K = mR * mR; g.batch = 1; g.kbatch = 1;
        g.A = q; g.lda = (int64_t)mR * mR; g.a_kcontig = true;
        g.B = W; g.ldb = stride_w; g.b_kcontig = true;
        g.C = c; g.ldc = n_right;
        err = gemm_split_k(ROT_FP64, g, split, s, "expect_pairs");
    }
    return err == hipSuccess ? ROT_OK : hip_fail(err, "rot_expect_cross");
}

rot_status rot_backward(const rot_problem* groups, int32_t n_groups, const void* const* dOut,
                        const int64_t* stride_dout, void* const* dO, void* const* dU, uint32_t flags,
                        rot_precision prec, void* workspace0, size_t workspace_bytes0, void* stream) {
    rot::TraceRange trace_("rot_backward");
    if (n_groups < 0 || (n_groups > 0 && (!groups || !dOut || !stride_dout)))
        return fail(ROT_ERR_INVALID_ARG, "null groups/dOut/stride_dout or negative n_groups");
    if (!valid_precision(prec)) return fail(ROT_ERR_INVALID_ARG, "unknown precision %d", (int)prec);
    if (flags & ~ROT_ASSUME_SYMMETRIC_O) return fail(ROT_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    const std::vector<rot_problem> rg = resolved_all(groups, n_groups);
    for (int gi = 0; gi < n_groups; gi++) {
        const rot_problem& p = rg[gi];
        rot_status st = validate_group(p, gi);
        if (st != ROT_OK) return st;
        if (p.n_ops == 0) continue;
        if (!dOut[gi]) return fail(ROT_ERR_INVALID_ARG, "group %d: null dOut", gi);
        if (stride_dout[gi] != 0 && stride_dout[gi] < (int64_t)p.mp * p.mp)
            return fail(ROT_ERR_INVALID_ARG, "group %d: stride_dout must be 0 or >= mp*mp", gi);
        if (prec == ROT_SPLIT_BF16 && !bf16_backward_supported(p.m, p.d, p.mp))
            return fail(ROT_ERR_UNSUPPORTED,
                        "group %d: split-bf16 adjoint operands must stay below 2 GiB (m=%d d=%d mp=%d); use ROT_FP32",
                        gi, p.m, p.d, p.mp);
    }
    const size_t min_ws = rot_workspace_size(groups, n_groups, prec, 1, 1);
    if (min_ws > 0) {
        if (!workspace0 || workspace_bytes0 < min_ws)
            return fail(ROT_ERR_WORKSPACE, "workspace %zu bytes < minimum %zu", workspace_bytes0, min_ws);
        if (reinterpret_cast<uintptr_t>(workspace0) % kAlign)
            return fail(ROT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t es = elem_size(prec);
    const bool sym = flags & ROT_ASSUME_SYMMETRIC_O;
    for (int gi = 0; gi < n_groups; gi++) {
        rot_problem p = rg[gi];
        void* dOg = dO ? dO[gi] : nullptr;
        void* dUg = dU ? dU[gi] : nullptr;
        if (p.n_ops == 0) {
            if (dUg) {
                hipError_t e = fill_zero(dUg, (int64_t)p.m * p.d * p.mp * es, s);
                if (e != hipSuccess) return hip_fail(e, "rot_backward zero dU");
            }
            continue;
        }
        if (!dOg && !dUg) continue;
        const int64_t md = (int64_t)p.m * p.d, tsz = md * p.mp;
        // U with padded rows is packed first: dO_b reads U_r (m x d*mp)
        const size_t ub = packed_u_bytes(p, prec);
        void* workspace = static_cast<char*>(workspace0) + ub;
        const size_t workspace_bytes = workspace_bytes0 - ub;
        if (ub) {
            hipError_t e = prof_timed("adj_pack_u", s, [&] {
                return hipMemcpy2DAsync(workspace0, (size_t)p.mp * es, p.U, (size_t)p.ldu * es, (size_t)p.mp * es,
                                        (size_t)md, hipMemcpyDeviceToDevice, s);
            });
            if (e != hipSuccess) return hip_fail(e, "rot_backward pack U");
            p.U = workspace0;
            p.ldu = p.mp;
        }
        if (prec == ROT_SPLIT_BF16) {
            int chunk = 1;
            while (chunk < p.n_ops && bf16_backward_workspace(p.m, p.d, p.mp, chunk + 1) <= workspace_bytes) chunk++;
            for (int b0 = 0; b0 < p.n_ops; b0 += chunk) {
                const int nb = std::min(chunk, p.n_ops - b0);
                hipError_t e = backward_bf16(p, b0, nb, static_cast<const float*>(dOut[gi]), stride_dout[gi],
                                             static_cast<float*>(dOg), static_cast<float*>(dUg), sym, workspace, s);
                if (e != hipSuccess) return hip_fail(e, "rot_backward split-bf16 launch");
            }
            continue;
        }
        const size_t per_op = t_bytes(p, prec);
        const size_t slots = workspace_bytes / per_op;
        // Chunk size, leaving `parts` slots for the partial dU sums when dU is
        // wanted and the workspace holds at least one operator per part.
        int parts = 0;
        if (dUg) {
            parts = du_split_parts(p, p.n_ops);
            while (parts > 1 && slots < (size_t)2 * parts) parts /= 2;
            if (parts < 2) parts = 0;
        }
        const int chunk = (int)std::min<size_t>((size_t)p.n_ops, slots - parts);
        const char* dout_base = static_cast<const char*>(dOut[gi]);
        const int64_t sd = stride_dout[gi];
        char* partial = static_cast<char*>(workspace) + (size_t)chunk * per_op;
        const int64_t part_stride = (int64_t)(per_op / es);
        for (int b0 = 0; b0 < p.n_ops; b0 += chunk) {
            const int nb = std::min(chunk, p.n_ops - b0);
            const void* g_b0 = dout_base + (size_t)b0 * sd * es;
            hipError_t e = hipSuccess;
            // P_b = U dOut_b ((m*d) x mp), the only intermediate: the adjoint of
            // stage 2 applied to dOut_b.  Viewed as P_b,r (m x d*mp) it gives
            // dO_b = P_b,r U_r^T, and dU_r = sum_b (O_b^T P_b,r + O_b Q_b,r)
            // with Q_b = U dOut_b^T, so stage 1 (O_b U_r) is never formed.
            auto form_P = [&](bool transposed, bool accumulate, const char* what) {
                GemmDesc a{};
                a.M = (int)md; a.N = p.mp; a.K = p.mp; a.batch = nb; a.kbatch = 1;
                a.A = p.U; a.lda = p.mp; a.a_bs = 0; a.a_kcontig = true;
                // B(alpha, beta) = dOut_b[alpha][beta], or dOut_b[beta][alpha] for Q_b
                a.B = g_b0; a.ldb = p.mp; a.b_bs = sd; a.b_kcontig = transposed;
                a.C = workspace; a.ldc = p.mp; a.c_bs = tsz; a.accumulate = accumulate;
                return gemm(prec, a, s, what);
            };
            e = form_P(false, false, "adj_P");
            if (dOg && e == hipSuccess) {
                GemmDesc b{};
                b.M = p.m; b.N = p.m; b.K = p.d * p.mp; b.batch = nb; b.kbatch = 1;
                b.A = workspace; b.lda = (int64_t)p.d * p.mp; b.a_bs = tsz; b.a_kcontig = true;
                b.B = p.U; b.ldb = (int64_t)p.d * p.mp; b.b_bs = 0; b.b_kcontig = true;
                b.C = static_cast<char*>(dOg) + (size_t)b0 * p.m * p.m * es; b.ldc = p.m;
                b.c_bs = (int64_t)p.m * p.m;
                e = gemm(prec, b, s, "adj_dO");
            }
            if (dUg && e == hipSuccess) {
                // The chunk's operators go to np parts of q operators each; the
                // remaining r operators are added to part 0.
                const int np = parts ? std::min(parts, nb) : 1;
                const int q = nb / np, r = nb % np;
                // dU_r (or its part) (+)= sum over the part's operators of A_b P_b,r,
                // A_b = O_b or O_b^T.
                auto reduce = [&](bool o_transposed, bool acc_first) -> hipError_t {
                    GemmDesc c{};
                    c.M = p.m; c.N = p.d * p.mp; c.K = p.m; c.batch = np; c.kbatch = q;
                    c.A = static_cast<const char*>(p.O) + (size_t)b0 * p.stride_o * es; c.lda = p.ldo;
                    c.a_ks = p.stride_o; c.a_bs = q * p.stride_o;
                    c.a_kcontig = !o_transposed;  // A(i, j) = O_b[i*ldo + j], or O_b[j*ldo + i]
                    c.B = workspace; c.ldb = (int64_t)p.d * p.mp; c.b_ks = tsz; c.b_bs = q * tsz;
                    c.b_kcontig = false;
                    c.C = np > 1 ? static_cast<void*>(partial) : dUg; c.ldc = (int64_t)p.d * p.mp;
                    c.c_bs = part_stride; c.accumulate = acc_first;
                    hipError_t err = gemm(prec, c, s, "adj_dU");
                    if (err == hipSuccess && r > 0) {
                        GemmDesc t = c;
                        t.batch = 1; t.kbatch = r; t.accumulate = true;
                        t.A = static_cast<const char*>(c.A) + (size_t)np * q * p.stride_o * es;
                        t.B = static_cast<const char*>(workspace) + (size_t)np * q * tsz * es;
                        err = gemm(prec, t, s, "adj_dU");
                    }
                    return err;
                };
                const bool first_acc = np == 1 && b0 > 0;
                if (sym) {
                    // O_b = O_b^T: dU_r = sum_b O_b (P_b + Q_b)_r
                    e = form_P(true, true, "adj_Q");
                    if (e == hipSuccess) e = reduce(false, first_acc);
                } else {
                    e = reduce(true, first_acc);
                    if (e == hipSuccess) e = form_P(true, false, "adj_Q");
                    if (e == hipSuccess) e = reduce(false, true);
                }
                if (e == hipSuccess && np > 1)
                    e = prof_timed("adj_dU_sum", s, [&] {
                        return sum_parts(dUg, partial, md * p.mp, np, part_stride, b0 > 0, prec == ROT_FP64, s);
                    });
            }
            if (e != hipSuccess) return hip_fail(e, "rot_backward launch");
        }
    }
    return ROT_OK;
}

size_t rot_pair_loss_workspace_size(int32_t mp, int32_t n_ops) {
    if (mp <= 0 || n_ops <= 0) return 0;
    return pair_loss_workspace_bytes(mp, n_ops);
}

rot_status rot_pair_loss(const void* X, int32_t mp, int32_t n_ops, int64_t stride_x, rot_precision prec,
                         const double* psi, double* loss, double* pairs, void* grad, void* workspace,
                         size_t workspace_bytes, void* stream) {
    rot::TraceRange trace_("rot_pair_loss");
    if (!valid_precision(prec)) return fail(ROT_ERR_INVALID_ARG, "unknown precision %d", (int)prec);
    if (mp <= 0 || n_ops <= 0 || n_ops > 65535)
        return fail(ROT_ERR_INVALID_ARG, "need mp > 0 and 0 < n_ops <= 65535");
    if (!X || !psi || !loss) return fail(ROT_ERR_INVALID_ARG, "null X, psi or loss");
    if (stride_x < (int64_t)mp * mp) return fail(ROT_ERR_INVALID_ARG, "stride_x < mp*mp");
    const size_t need = pair_loss_workspace_bytes(mp, n_ops);
    if (!workspace || workspace_bytes < need)
        return fail(ROT_ERR_WORKSPACE, "workspace %zu bytes < minimum %zu", workspace_bytes, need);
    hipError_t e = pair_loss(X, mp, n_ops, stride_x, prec == ROT_FP64, psi, loss, pairs, grad, workspace,
                             static_cast<hipStream_t>(stream));
    return e == hipSuccess ? ROT_OK : hip_fail(e, "rot_pair_loss launch");
}

size_t rot_isometry_workspace_size(int32_t rows, int32_t cols, rot_precision prec) {
    if (rows <= 0 || cols <= 0 || !valid_precision(prec)) return 0;
    return isometry_workspace_bytes(rows, cols, prec == ROT_FP64);
}

rot_status rot_check_isometry(const void* U, int32_t rows, int32_t cols, int64_t ldu, rot_precision prec,
                              double tol, double* max_dev_host, void* workspace, size_t workspace_bytes,
                              void* stream) {
    rot::TraceRange trace_("rot_check_isometry");
    if (!valid_precision(prec)) return fail(ROT_ERR_INVALID_ARG, "unknown precision %d", (int)prec);
    if (!U || !max_dev_host || rows <= 0 || cols <= 0 || cols > rows)
        return fail(ROT_ERR_INVALID_ARG, "need U, max_dev_host and 0 < cols <= rows");
    if (ldu == 0) ldu = cols;
    if (ldu < cols || ldu > INT32_MAX) return fail(ROT_ERR_INVALID_ARG, "ldu %lld must be >= cols", (long long)ldu);
    const size_t need = isometry_workspace_bytes(rows, cols, prec == ROT_FP64);
    if (!workspace || workspace_bytes < need)
        return fail(ROT_ERR_WORKSPACE, "workspace %zu bytes < minimum %zu", workspace_bytes, need);
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(ROT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* ws = static_cast<double*>(workspace);
    hipError_t e = isometry_deviation(U, rows, cols, ldu, prec == ROT_FP64, ws, s);
    if (e == hipSuccess) e = hipMemcpyAsync(max_dev_host, ws, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "rot_check_isometry");
    if (!(*max_dev_host <= tol))
        return fail(ROT_ERR_NOT_ISOMETRY, "max|U^T U - I| = %.3e exceeds tol %.3e", *max_dev_host, tol);
    return ROT_OK;
}

namespace {
constexpr int kDmMaxStates = 4096;

rot_status validate_dm(const rot_dm_sector* sectors, int32_t n_sectors) {
    if (!sectors || n_sectors <= 0) return fail(ROT_ERR_INVALID_ARG, "sectors is null or n_sectors <= 0");
    for (int k = 0; k < n_sectors; k++) {
        const rot_dm_sector& s = sectors[k];
        if (s.n < 1 || s.n > kDmMaxStates)
            return fail(ROT_ERR_INVALID_ARG, "sector %d: n = %d outside 1..%d", k, s.n, kDmMaxStates);
        if (s.r < 0) return fail(ROT_ERR_INVALID_ARG, "sector %d: negative r", k);
        if (s.r > 0 && (!s.psi || s.ld_psi < s.r))
            return fail(ROT_ERR_INVALID_ARG, "sector %d: null psi or ld_psi < r", k);
        if (!s.w || !s.V || s.ld_v < s.n) return fail(ROT_ERR_INVALID_ARG, "sector %d: null w or V, or ld_v < n", k);
    }
    return ROT_OK;
}
}  // namespace

size_t rot_density_workspace_size(const rot_dm_sector* sectors, int32_t n_sectors) {
    if (validate_dm(sectors, n_sectors) != ROT_OK) return 0;
    return density_workspace_bytes(sectors, n_sectors);
}

rot_status rot_density_basis(const rot_dm_sector* sectors, int32_t n_sectors, int64_t m_keep, int32_t* kept,
                             double* eps, void* workspace, size_t workspace_bytes, void* stream) {
    rot::TraceRange trace_("rot_density_basis");
    const rot_status v = validate_dm(sectors, n_sectors);
    if (v != ROT_OK) return v;
    if (m_keep < 0) return fail(ROT_ERR_INVALID_ARG, "m_keep must be >= 0");
    if (!kept || !eps) return fail(ROT_ERR_INVALID_ARG, "null kept or eps");
    const size_t need = density_workspace_bytes(sectors, n_sectors);
    if (!workspace || workspace_bytes < need)
        return fail(ROT_ERR_WORKSPACE, "workspace %zu bytes < minimum %zu", workspace_bytes, need);
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(ROT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    bool converged = false;
    const hipError_t e = density_basis(sectors, n_sectors, m_keep, kept, eps, workspace,
                                       static_cast<hipStream_t>(stream), &converged);
    if (e != hipSuccess) return hip_fail(e, "rot_density_basis");
    if (!converged) return fail(ROT_ERR_NOT_CONVERGED, "Jacobi sweeps exhausted before every sector converged");
    return ROT_OK;
}

rot_status rot_split_bf16(const float* x, int64_t n, uint16_t* hi, uint16_t* lo, void* stream) {
    rot::TraceRange trace_("rot_split_bf16");
    if (n < 0 || (n > 0 && (!x || !hi || !lo))) return fail(ROT_ERR_INVALID_ARG, "null buffer or n < 0");
    if (n == 0) return ROT_OK;
    hipError_t e = split_bf16(x, n, hi, lo, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? ROT_OK : hip_fail(e, "rot_split_bf16 launch");
}

size_t rot_blocked_workspace_size(const rot_blocked_problem* p) {
    std::string why;
    if (!p || blocked_validate(p, &why) != ROT_OK) return 0;
    return blocked_workspace_bytes(p);
}

rot_status rot_batch_blocked(const rot_blocked_problem* p, rot_precision prec, void* workspace,
                             size_t workspace_bytes, void* stream) {
    rot::TraceRange trace_("rot_batch_blocked");
    if (!p) return fail(ROT_ERR_INVALID_ARG, "null problem");
    if (prec != ROT_FP32) return fail(ROT_ERR_UNSUPPORTED, "rot_batch_blocked supports ROT_FP32 only");
    std::string why;
    rot_status st = blocked_validate(p, &why);
    if (st != ROT_OK) return fail(st, "%s", why.c_str());
    const size_t need = blocked_workspace_bytes(p);
    if (need > 0 && (!workspace || workspace_bytes < need))
        return fail(ROT_ERR_WORKSPACE, "workspace %zu bytes < minimum %zu", workspace_bytes, need);
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(ROT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    hipError_t e = rotate_blocked(p, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
    if (e == hipErrorStreamCaptureUnsupported) return ROT_ERR_UNSUPPORTED;  // message already set
    return e == hipSuccess ? ROT_OK : hip_fail(e, "rot_batch_blocked");
}

}  // extern "C"
