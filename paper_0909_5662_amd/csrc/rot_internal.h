// Internal declarations of librot (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

#include "librot.h"

namespace rot {

// Batched, K-batched GEMM on row-major operands:
//   C[g] (M x N) (+)= alpha_sign * sum_{kb < kbatch} A[g,kb] (M x K) * B[g,kb] (K x N)
// Operand layouts:
//   a_kcontig: A(m,k) at A[m*lda + k]   else A(m,k) at A[k*lda + m]
//   b_kcontig: B(k,n) at B[n*ldb + k]   else B(k,n) at B[k*ldb + n]
// Element (batch g, k-batch kb) bases: A + g*a_bs + kb*a_ks (same for B).
// C[g] at C + g*c_bs with leading dimension ldc.  accumulate: C += result.
struct GemmDesc {
    int M, N, K;
    int batch, kbatch;
    const void* A;
    int64_t lda, a_bs, a_ks;
    const void* B;
    int64_t ldb, b_bs, b_ks;
    void* C;
    int64_t ldc, c_bs;
    bool a_kcontig, b_kcontig, accumulate;
    // symmetric output (M == N, no accumulation): only tiles on or above the
    // diagonal are computed, each off-diagonal one also stored transposed
    bool upper;
    // split K (parts > 1; kbatch == 1, no upper, no accumulate): part p
    // multiplies K range [p*kp, min(K, (p+1)*kp)) and writes its product to
    // C + p*c_ps; the caller adds the parts
    int parts, kp;
    int64_t c_ps;
};

// ---- grouped GEMM over a work-list (grouped.hip) ----
// k128d: 128 x 128 tiles whose K slices are filled by buffer loads with LDS
// destination (every problem of the launch must carry kGroupedWhole).
enum class GroupedShape : int { k128 = 0, k64 = 1, k32 = 2, k128d = 3 };
constexpr int kGroupedVec = 1;         // 16-byte vector loads allowed for this problem
constexpr int kGroupedAccumulate = 2;  // C += result
// Whole 128 x 128 tiles and 16-wide K slices, 16-byte aligned rows, no
// accumulation, and every byte offset of A and B (from the problem's
// positions) below 2^32.
constexpr int kGroupedWhole = 4;
// One GEMM C (M x N) (+)= A (M x K) B (K x N); operand/result positions are
// element offsets from the launch's base pointers (absolute byte addresses
// when the base is null).  Layouts are per launch.
struct GroupedProblem {
    int M, N, K, flags;
    int64_t a_off, lda, b_off, ldb, c_off, ldc;
};
struct GroupedTile {
    int prob, m0, n0, pad;
};
struct GroupedLaunch {
    const float* a_base;
    const float* b_base;
    float* c_base;
    const GroupedProblem* probs;  // device
    const GroupedTile* tiles;     // device
    int n_tiles;
    bool a_kcontig, b_kcontig;    // as in GemmDesc
    bool dynamic;                 // atomic tile queue (needs counter) vs static stride
    GroupedShape shape;
    int grid;                     // persistent workgroups (<= 0: one per tile)
    int* counter;                 // device int for the dynamic queue
};
int grouped_tile_edge(GroupedShape shape);
hipError_t grouped_gemm_f32(const GroupedLaunch& L, hipStream_t stream);

// Records `msg` as the calling thread's last error (rot_last_error) and
// returns `s`.
rot_status set_error(rot_status s, const char* msg);

// Tuning cache (tune_cache.cpp): key -> tokens, in memory and in the file
// named by ROT_TUNE_CACHE.
bool tune_get(const std::string& key, std::vector<std::string>* tokens);
void tune_put(const std::string& key, const std::vector<std::string>& tokens);

// Environment switches (env.cpp): ROT_LOG_LEVEL, ROT_TRACE, ROT_DISABLE_GRAPH,
// ROT_SCHEDULE.
int log_level();
void log_msg(int level, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
bool graphs_disabled();
int forced_schedule();  // -1 none, 0 static, 1 dynamic
// roctx range around an entry point while ROT_TRACE is set
class TraceRange {
   public:
    explicit TraceRange(const char* name);
    ~TraceRange();
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;

   private:
    bool active_ = false;
};

// Runs `launch` (which enqueues kernels on `stream`); when per-kernel timing
// is enabled (rot_profile_enable) it is bracketed by HIP events recorded on
// `stream` and filed under `name`.
hipError_t prof_timed(const char* name, hipStream_t stream, const std::function<hipError_t()>& launch);

// Enqueue on `stream`; returns hipSuccess or the launch error.
constexpr int kGemmTile = 128;  // output tile edge of gemm_f32 / gemm_f64
hipError_t gemm_f32(const GemmDesc& g, hipStream_t stream);
hipError_t gemm_f64(const GemmDesc& g, hipStream_t stream);

// Split-BF16 launch configuration (gemm_bf16x3.hip): tile edge 256 (eight
// waves of 128 x 64) or 128 (four waves of 64 x 64), LDS ring depth 4 or 5,
// tile order (0: M tiles fastest per batch element; -1: N tiles fastest;
// G > 0: groups of G M tiles across all columns); and the choice of the two
// rotation stages for one shape.
struct Bf16Cfg {
    int tile = 256, ring = 4, order = 0;
    int direct = 0;  // 1: B fragments straight from global memory (256 x 256 tiles only)
};
struct Bf16Choice {
    Bf16Cfg s1, s2;
};

// FP64 rotation of small blocks (m, m' <= 64) in one launch (small.hip).
bool rotate_small_f64_applies(const rot_problem& p);
hipError_t rotate_small_f64(const rot_problem& p, hipStream_t stream);

// Zero `bytes` bytes with a fill kernel (safe under stream capture).
hipError_t fill_zero(void* p, int64_t bytes, hipStream_t stream);

// Superblock measurements (measure.hip): e_b = sum_e Z_b[e] rho[e] in FP64
// (n elements per operator, fixed summation order; partial needs
// expect_dot_scratch(n_ops) bytes), and q_b = partial trace of Q_b over the
// right site (Q_b of side dR*mR at Q + b*q_stride, q_b of side mR).
size_t expect_dot_scratch(int n_ops);
hipError_t expect_dots(const void* Z, bool z_double, int64_t stride_z, int64_t n, int n_ops, const double* rho,
                       double* partial, double* e, hipStream_t s);
hipError_t partial_trace(const double* Q, int64_t q_stride, int mR, int dR, int n_ops, double* q, hipStream_t s);

// A d x d site operator passed by value to kernels (d <= kMaxSite).
constexpr int kMaxSite = 16;
struct SiteMatrix {
    double v[kMaxSite * kMaxSite];  // row-major S[s][t] at v[s*d + t]
};
// Up = (diag(x) (x) S^T) U for U with m*d rows of mp (x may be null: identity).
hipError_t site_mix(const void* U, int m, int d, int mp, const SiteMatrix& S, const void* x, void* Up,
                    bool is_double, hipStream_t stream);
// dst[b] (rows x cols, row stride ld, matrix stride bs; nmat matrices) =
// sum over p of the packed matrices at src + p*pstride, in ascending p.
hipError_t sum_parts_2d(void* dst, int64_t ld, int64_t bs, const void* src, int rows, int cols, int nmat, int parts,
                        int64_t pstride, bool is_double, hipStream_t stream);
// dst (+)= sum of `parts` arrays of n elements at src + p*stride, summed in
// ascending p (deterministic).
hipError_t sum_parts(void* dst, const void* src, int64_t n, int parts, int64_t stride, bool accumulate,
                     bool is_double, hipStream_t stream);

// FP64 reductions (reduce_f64.hip).
size_t pair_loss_workspace_bytes(int mp, int n_ops);
hipError_t pair_loss(const void* X, int mp, int n_ops, int64_t stride, bool is_double,
                     const double* psi, double* loss, double* pairs, void* grad, void* ws,
                     hipStream_t stream);
size_t isometry_workspace_bytes(int64_t rows, int cols, bool is_double);
// Result (max |U^T U - I|) lands in ws[0] (device).
hipError_t isometry_deviation(const void* U, int rows, int cols, int64_t ldu, bool is_double, double* ws,
                              hipStream_t stream);

}  // namespace rot
