/*
 * librot: batched density-matrix rotation of stored operators on one
 * AMD Instinct MI355X (gfx950).
 *
 * Operation (Rincon, Garcia & Hallberg, "Improved parallelization techniques
 * for the density matrix renormalization group", Sec. 2 step 5 and the
 * paragraph that follows the step list; Sec. 3.2): every operator Z stored
 * on the block B is blocked onto the enlarged block [B a] (tensored with the
 * identity of the added site) and then rotated and decimated with the
 * truncation matrix R built from the kept density-matrix eigenvectors,
 * Z_new = R Z_[B a] R^+.  In this library, with real arithmetic:
 *
 *     out_b = U^T (O_b (x) I_d) U           for every operator b of a group,
 *
 * where U = R^T is the (m*d) x mp isometry whose columns are the kept
 * eigenvectors, with block-site row index r = i*d + s (old block state i
 * slow, site state s fast).  The Kronecker product is never formed: stage 1
 * computes T_b = O_b * U_r with U_r the m x (d*mp) view of U (the paper's
 * "Z R^+" first), stage 2 computes out_b = U^T T_b ("R (Z R^+)").
 *
 * Conventions for every entry point:
 *  - All matrices are dense and row-major.  Data pointers are device
 *    pointers unless the argument says "host".  FP64 precision takes double
 *    buffers; FP32 and split-BF16 take float buffers.
 *  - The caller allocates and owns every buffer, including the workspace;
 *    the library keeps no pointer after a call returns.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *    default stream).  Argument errors are detected on the host before any
 *    launch and returned synchronously; nothing aborts or throws.
 *  - A status other than ROT_OK leaves the outputs unspecified;
 *    rot_last_error() then describes the failure (per calling thread).
 */
#ifndef LIBROT_H
#define LIBROT_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define ROT_API __attribute__((visibility("default")))
#else
#define ROT_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ROT_OK = 0,
    ROT_ERR_INVALID_ARG = -1,   /* null pointer, bad size or stride, bad table */
    ROT_ERR_UNSUPPORTED = -2,   /* valid request this library does not implement */
    ROT_ERR_WORKSPACE = -3,     /* workspace smaller than the minimum */
    ROT_ERR_HIP = -4,           /* HIP runtime error (launch, device query) */
    ROT_ERR_NOT_ISOMETRY = -5,  /* rot_check_isometry: max|U^T U - I| above tolerance */
    ROT_ERR_NOT_CONVERGED = -6  /* rot_density_basis: Jacobi sweeps exhausted */
} rot_status;

typedef enum {
    ROT_FP64 = 0,        /* double buffers, FP64 matrix cores */
    ROT_FP32 = 1,        /* float buffers, FP32 matrix cores, FP32 accumulation */
    ROT_SPLIT_BF16 = 2   /* float buffers; each operand x = hi + lo with
                            hi = bf16(x), lo = bf16(x - hi) (round to nearest
                            even); products hi*hi + hi*lo + lo*hi on BF16
                            matrix cores, FP32 accumulation */
} rot_precision;

/*
 * One group of operators sharing one truncation matrix (Sec. 3.2: R is
 * common to all stored operators of a step).
 *   m      old block dimension (> 0)
 *   d      added-site dimension (> 0; 4 for the Hubbard chain of Eq. (4))
 *   mp     number of kept states (0 < mp <= m*d)
 *   n_ops  number of operators (>= 0; 0 is a no-op)
 *   U      (m*d) x mp, row r = i*d + s, element (r, a) at U[r*ldu + a];
 *          ldu >= mp (0 selects mp)
 *   O      operator b is the m x m matrix at O + b*stride_o, element (i, j)
 *          at [i*ldo + j]; ldo >= m (0 selects m); stride_o >= (m-1)*ldo + m
 *   out    result b is the mp x mp matrix at out + b*stride_out, element
 *          (a, c) at [a*ldout + c]; ldout >= mp (0 selects mp); stride_out
 *          >= (mp-1)*ldout + mp; must not overlap U or O.  Only the mp
 *          entries of each row are written: padding between rows is kept.
 * All leading dimensions and strides are in elements.  16-byte aligned
 * pointers with leading dimensions and strides that are multiples of 4
 * (FP32) or 2 (FP64) take the vector load paths; any other layout is
 * accepted and read element by element at the edges of each tile.
 */
typedef struct {
    int32_t m, d, mp, n_ops;
    const void* U;
    int64_t ldu;
    const void* O;
    int64_t ldo, stride_o;
    void* out;
    int64_t ldout, stride_out;
} rot_problem;

/*
 * Dense rotation of one or more groups: out_b = U^T (O_b (x) I_d) U.
 * Sec. 2 step 5; Sec. 3.2 (order of the two products; all stored Z_i and
 * Z_i Z_j of a step share R).
 * workspace: device memory of at least rot_workspace_size(..., 1) bytes,
 * 256-byte aligned; operators are processed in chunks that fit it (larger
 * workspaces give larger, faster chunks).  When a group's stage-2 output has
 * few tiles (fewer than 256 of 128 x 128) and the workspace holds the whole
 * group with rot_workspace_size(..., 0)'s room for partial sums, FP32 and
 * FP64 stage 2 is split over K into parts added in a fixed order: results
 * are deterministic for a given workspace size but may differ in the last
 * bits from a call whose workspace is too small to split.  An FP64 group
 * with m <= 64 and mp <= 64 (not ROT_OUT_SYMMETRIC) is rotated in a single
 * launch that keeps both stages in LDS and leaves the workspace untouched
 * (its size is still checked as for any group).  Groups may have
 * different m, d, mp.  ROT_SPLIT_BF16 picks each stage's tile configuration per shape (m, d,
 * mp, chunk): from the tuning cache (in memory, and in the file named by
 * ROT_TUNE_CACHE), else on the shape's first call by timing the candidates
 * on the first chunk, which synchronises `stream` once (not under stream
 * capture, nor with ROT_AUTOTUNE=0: the defaults are used then); every
 * configuration gives the same bits.  Returns ROT_OK, ROT_ERR_INVALID_ARG,
 * ROT_ERR_WORKSPACE, ROT_ERR_HIP.
 */
ROT_API rot_status rot_batch(const rot_problem* groups, int32_t n_groups, rot_precision prec,
                     void* workspace, size_t workspace_bytes, void* stream);

#define ROT_ASSUME_SYMMETRIC_O 1u

/*
 * rot_batch with flags (same arguments otherwise; rot_batch is flags = 0).
 * ROT_ASSUME_SYMMETRIC_O: every O_b is symmetric, so every out_b is
 * symmetric (U^T (O (x) I) U with O = O^T); stage 2 computes only the output
 * tiles on and above the diagonal and stores each off-diagonal tile also
 * transposed: 2 m^2 d m' + about m d m'^2 (1 + 128/m') flops per operator
 * instead of 2 m^2 d m' + 2 m d m'^2.  out_b is then exactly symmetric; for non-symmetric O_b
 * the result is wrong (only the upper triangle of U^T (O (x) I) U is kept).
 */
ROT_API rot_status rot_batch_ex(const rot_problem* groups, int32_t n_groups, rot_precision prec, uint32_t flags,
                        void* workspace, size_t workspace_bytes, void* stream);

/*
 * rot_batch_ex without a workspace argument, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid allocation).  The workspace is a fixed device array
 * of rot_noalloc_scratch_bytes() bytes (128 MiB) inside the library: each GPU
 * the library runs on holds its own copy until the process ends.  The call
 * allocates nothing (its first call on a device looks the array's address
 * up once).  Groups whose single-operator workspace (rot_workspace_size with
 * ops_per_chunk = 1) exceeds the array return ROT_ERR_WORKSPACE; smaller ones
 * run in operator chunks that fit it.  Every call on one GPU shares that
 * GPU's array: calls that overlap in time on one GPU (other streams, other
 * threads) race and must be serialised by the caller; calls on one stream
 * are ordered and safe.  Results equal rot_batch_ex's for the same chunking.
 */
ROT_API rot_status rot_batch_noalloc(const rot_problem* groups, int32_t n_groups, rot_precision prec, uint32_t flags,
                                     void* stream);
ROT_API size_t rot_noalloc_scratch_bytes(void);

/*
 * Workspace bytes needed by rot_batch / rot_backward for these groups when
 * up to `ops_per_chunk` operators are processed at once (<= 0: all
 * operators of the largest group).  `for_backward` != 0 sizes it for
 * rot_backward: the chunk's intermediates plus, when dU has fewer than
 * 1024 output tiles of 128x128, up to 8 partial sums of dU (the operator sum
 * is split into parts that run concurrently and are added in fixed order).
 * rot_backward accepts any workspace of at least the ops_per_chunk = 1 size
 * and uses fewer parts, or none, when it is smaller.  Returns 0 for invalid
 * arguments.
 */
ROT_API size_t rot_workspace_size(const rot_problem* groups, int32_t n_groups, rot_precision prec,
                          int32_t ops_per_chunk, int32_t for_backward);

/*
 * Reverse-mode derivative of rot_batch (not in the paper).  For each group,
 * given dOut_b = dL/dout_b (mp x mp at dOut[g] + b*stride_dout[g]; a stride
 * of 0 broadcasts one matrix to every operator) it writes
 *   dO_b = sum_s U_s dOut_b U_s^T     (m x m at dO[g] + b*m*m), U_s the rows
 *                                      s, s+d, s+2d, ... of U
 *   dU   = sum_b [ (O_b (x) I) U dOut_b^T + (O_b^T (x) I) U dOut_b ]
 *                                     ((m*d) x mp at dU[g], summed over b)
 * Nothing is kept from the forward call: with P_b = U dOut_b and
 * Q_b = U dOut_b^T (viewed as m x d*mp), dO_b = P_b U_r^T and
 * dU = sum_b O_b^T P_b + O_b Q_b, so the stage-1 intermediate is never
 * formed.  dO, dU (host arrays of n_groups device pointers) may be NULL, and
 * so may any element, to skip that output.  flags: ROT_ASSUME_SYMMETRIC_O
 * merges the two dU terms into sum_b O_b (P_b + Q_b) (valid only when every
 * O_b is symmetric): four products of 2 m^2 d mp flops per operator instead
 * of five.
 * Summation order is fixed: results are deterministic.
 */
ROT_API rot_status rot_backward(const rot_problem* groups, int32_t n_groups,
                        const void* const* dOut, const int64_t* stride_dout,
                        void* const* dO, void* const* dU, uint32_t flags, rot_precision prec,
                        void* workspace, size_t workspace_bytes, void* stream);

/*
 * Operators blocked together with the added site (Sec. 2 step 3: the blocking
 * Z_[B a] <- Z_[B (+) a] for operators that act on the new site a; Sec. 3.2
 * task ii), rotated as in step 5:
 *     out_b = U^T (X_b (x) S) U          (mp x mp at out + b*stride_out)
 * S is one d x d site operator for the group (host memory, d*d doubles,
 * row-major, d <= 16); X_b acts on the old block, by block_kind:
 *   ROT_BLOCK_IDENTITY  X = I_m, the site's own operator I_B (x) Z_a
 *                       (n_ops = 1, X = NULL);
 *   ROT_BLOCK_DIAGONAL  X = diag(x), x = m values at X: with x the block's
 *                       fermion parity P_B = (-1)^N_B this is a fermionic site
 *                       operator with its Jordan-Wigner string (n_ops = 1);
 *   ROT_BLOCK_DENSE     X_b = m x m at X + b*stride_x (stride_x >= m*m): the
 *                       block-site products Z_B (x) Z_a, including the
 *                       hopping-type c+_B P_B (x) c_a (n_ops >= 0).
 * U and out follow rot_problem (U (m*d) x mp, row r = i*d + s).  X (x) S is
 * never formed: with U' = (diag(x) (x) S^T) U, out = U'^T U for the identity
 * and diagonal kinds and out = U'^T (X_b U_r) for the dense kind.
 * Precisions ROT_FP64 and ROT_FP32 (buffers of that type; S is always
 * double).  workspace: at least rot_site_workspace_size(..., 1) bytes,
 * 256-byte aligned; larger workspaces give larger operator chunks.
 */
#define ROT_BLOCK_IDENTITY 0
#define ROT_BLOCK_DIAGONAL 1
#define ROT_BLOCK_DENSE 2
typedef struct {
    int32_t m, d, mp, n_ops;
    int32_t block_kind;
    const void* U;
    const double* site;
    const void* X;
    int64_t stride_x;
    void* out;
    int64_t stride_out;
} rot_site_problem;

ROT_API size_t rot_site_workspace_size(const rot_site_problem* groups, int32_t n_groups, rot_precision prec,
                               int32_t ops_per_chunk);
ROT_API rot_status rot_batch_site(const rot_site_problem* groups, int32_t n_groups, rot_precision prec,
                          void* workspace, size_t workspace_bytes, void* stream);

/*
 * Measurements in the superblock state (Sec. 3.2: <Z_i> = <psi0|Z_i|psi0> and
 * <Z_i Z_j>, with correlations between the two blocks taken as products of
 * operators of each block).  psi is the state of [B a a~ B~] as a matrix
 * (FP64, device, row-major): row i*d + s (state i of block B, state s of
 * site a), column s'*mR + j (state s' of site a~, state j of block B~).
 *
 * rot_expect_block: e_b = <psi| Z_b (x) I |psi> for n_ops operators Z_b of
 *   block B (m x m at Z + b*stride_z, stride_z >= m*m; FP64 or FP32 by prec),
 *   the stored Z_i and Z_i Z_j alike, written to e (n_ops doubles, device).
 *   psi has m*d rows of ncols columns.  Computed as <Z_b, rho_B> with rho_B
 *   the reduced density matrix of B (one FP64 product of psi with itself),
 *   then FP64 dot products summed in a fixed order.  workspace:
 *   rot_expect_block_workspace_size(m, d, ncols, n_ops) bytes, 256-byte
 *   aligned.
 * rot_expect_cross: c[b*n_right + k] = <psi| (Z_b (x) I_a) (x) (I_a~ (x) W_k) |psi>
 *   for Z_b on B (m x m, FP64, stride_z >= m*m) and W_k on B~ (mR x mR, FP64,
 *   stride_w >= mR*mR); psi is (m*d) x (dR*mR); c (n_left*n_right doubles)
 *   on the device.  Computed as <q_b, W_k> with q_b the partial trace over
 *   a~ of psi^T (Z_b (x) I_d) psi (the rotation of Z_b with psi in place of U,
 *   FP64), then one FP64 product over all pairs.  workspace:
 *   rot_expect_cross_workspace_size(m, d, mR, dR, n_left, n_right,
 *   ops_per_chunk) bytes (ops_per_chunk left operators per chunk, <= 0: all;
 *   at least 1).  Products whose outputs have few tiles are split over K
 *   into partial sums added in a fixed order, so results do not depend on
 *   the chunking.
 * Both return ROT_OK, ROT_ERR_INVALID_ARG, ROT_ERR_WORKSPACE or ROT_ERR_HIP.
 */
ROT_API size_t rot_expect_block_workspace_size(int32_t m, int32_t d, int64_t ncols, int32_t n_ops);
ROT_API rot_status rot_expect_block(const double* psi, int32_t m, int32_t d, int64_t ncols, const void* Z,
                            int32_t n_ops, int64_t stride_z, rot_precision prec, double* e, void* workspace,
                            size_t workspace_bytes, void* stream);
ROT_API size_t rot_expect_cross_workspace_size(int32_t m, int32_t d, int32_t mR, int32_t dR, int32_t n_left,
                                       int32_t n_right, int32_t ops_per_chunk);
ROT_API rot_status rot_expect_cross(const double* psi, int32_t m, int32_t d, int32_t mR, int32_t dR,
                            const double* Z, int32_t n_left, int64_t stride_z, const double* W,
                            int32_t n_right, int64_t stride_w, double* c, void* workspace,
                            size_t workspace_bytes, void* stream);

/*
 * Plans: repeated rotation of a fixed set of groups with different sizes (a
 * sweep step rotates the stored operators of many blocks; Sec. 3.2 counts
 * l(l+3)/2 of them per block).  rot_plan_create buckets the groups into size
 * classes (ceil log2 of m*d and of mp), packs their operators into chunks
 * whose stage-1 intermediates fit `workspace`, builds per-chunk work-lists for
 * a grouped persistent kernel, picks per class the tile shape and the
 * schedule (static contiguous runs, like the paper's uniform-matrix
 * distribution, or an atomic tile queue, like its pool of tasks) from the
 * tuning cache or by timing candidates on the class's first chunk, and
 * captures all launches in a hipGraph.  Only ROT_FP32.
 *   groups, workspace: as for rot_batch; every buffer (U, O, out, workspace)
 *       is bound to the plan by address and must stay valid, unmoved and
 *       unoverlapped until rot_plan_destroy or until rot_plan_rebind binds
 *       other U, O and out buffers.
 *   stream: pending work on it is waited for before tuning writes to out and
 *       the workspace; create returns after its own device work has finished.
 *   flags: ROT_PLAN_NO_GRAPH (issue launches directly on execute),
 *       ROT_PLAN_NO_TUNE (use cache entries or the default, never time),
 *       ROT_PLAN_RETUNE (time candidates even when the cache has an entry).
 *   The tuning cache lives in memory and, when the environment variable
 *   ROT_TUNE_CACHE names a file, in that text file (unreadable lines are
 *   ignored).  Plans own device memory for their work-lists, a stream and the
 *   graph; they are not thread-safe (one caller at a time per plan).
 * rot_plan_execute enqueues one full rotation of every group on `stream`.
 * rot_plan_describe writes a JSON summary (classes, choices) into buf and
 * returns its full length (-1 for a null plan).
 */
typedef struct rot_plan_s* rot_plan;
#define ROT_PLAN_NO_GRAPH 1u
#define ROT_PLAN_NO_TUNE 2u
#define ROT_PLAN_RETUNE 4u
ROT_API rot_status rot_plan_create(const rot_problem* groups, int32_t n_groups, rot_precision prec,
                                   void* workspace, size_t workspace_bytes, uint32_t flags,
                                   void* stream, rot_plan* plan);
ROT_API rot_status rot_plan_execute(rot_plan plan, void* stream);
/*
 * rot_plan_rebind: point the plan at new U, O and out buffers (a DMRG step
 * rotates the same shapes with new data; Sec. 3.2).  groups must match the
 * plan's groups one by one in m, d, mp, n_ops, leading dimensions and
 * strides; the workspace stays bound.  The plan's work-list descriptors are
 * recomputed on the host and copied into its device tables on `stream`, so
 * executions enqueued on `stream` before the rebind use the old buffers and
 * those after it the new ones (graph, tiles and tuned choices are kept: no
 * capture or tuning is repeated).  An execution in flight on another stream
 * must be ordered against the rebind by the caller.  The first rebind
 * allocates a pinned staging buffer; each rebind waits for the previous
 * rebind's copies to leave it.  A size class tuned to the kernel that copies
 * K slices straight into LDS (all its products in whole 128 x 128 tiles with
 * 16-byte aligned U and O) keeps that kernel: new U or O buffers of such a
 * class that are not 16-byte aligned are refused with ROT_ERR_INVALID_ARG
 * before anything changes.
 */
ROT_API rot_status rot_plan_rebind(rot_plan plan, const rot_problem* groups, int32_t n_groups, void* stream);
ROT_API int32_t rot_plan_describe(rot_plan plan, char* buf, size_t len);
ROT_API rot_status rot_plan_destroy(rot_plan plan);

/*
 * Quantum-number (N_up, N_down) block-sparse rotation, Eq. (10) and the
 * paragraph after it: operators and U are block-sparse by particle numbers;
 * an operator with shift Delta maps old sector q to q + Delta (Delta = (0,0)
 * for number-conserving operators such as n and S^z, (1,0) or (0,1) for
 * c^+_up, c^+_dn).  For every operator and kept sector Q with Q + Delta kept:
 *   out(Q+Delta <- Q) = sum_s U_{Q+Delta}[s-rows]^T O(q_s+Delta <- q_s) U_Q[s-rows],
 * q_s = Q - qn(s); terms whose sectors are absent are zero.
 *
 * All tables are host arrays; block data are device arrays of floats.
 *   site_qn      d pairs (n_up, n_dn) of the site states
 *   old_sec      n_old sectors {n_up, n_dn, dim, offset} of the old block
 *                (dims sum to m; offsets are their prefix sums)
 *   new_sec      n_new kept sectors (dims sum to mp)
 *   U_blk/U_off  U_Q for new sector k is the M_k x new_sec[k].dim matrix at
 *                U_blk + U_off[k]; its rows run over s ascending and, inside,
 *                over the old states of sector Q - qn(s) (absent sectors give
 *                no rows), so M_k = sum_s dim(Q - qn(s))
 *   shift        n_ops pairs Delta
 *   O_blk/O_off  block (q+Delta <- q) of operator b for old sector k is the
 *                dim(q+Delta) x dim(q) matrix at O_blk + O_off[b*n_old + k];
 *                -1 means the block is absent (zero)
 *   out_blk/out_off  block (Q+Delta <- Q) of operator b for new sector k is
 *                written at out_blk + out_off[b*n_new + k] (dim(Q+Delta) x
 *                dim(Q)); -1 means not requested.  A requested block whose
 *                target sector is not kept is an error.
 * Only ROT_FP32 is supported.  workspace: at least
 * rot_blocked_workspace_size(p) bytes; it also holds the call's tile-queue
 * counter, so calls on different streams with different workspaces are
 * independent (one workspace must not serve two calls in flight).  The first
 * call for a block structure (sector tables, offsets and buffer alignment)
 * builds its work-lists in library-owned device memory, times the available
 * execution paths (one fused kernel in two register layouts, its variant
 * that loads whole row blocks of operator rows, two grouped launches, or two
 * launches that stack each shift's operators into one product per sector
 * combination; that one applies while no kept sector has more than four
 * site-state segments and each shift's intermediates for one kept sector stay
 * under 1 GiB) and keeps the fastest for later calls with the same
 * structure; every call's result comes from the kept path, so repeated calls
 * agree bit for bit.  ROT_BLOCKED_PATH=fused|fused_wide|rowblock|
 * rowblock_wide|grouped|stacked in the environment forces one.  Work-lists are cached for the 8 most recently used structures;
 * a structure used while `stream` is being captured into a graph is kept for
 * the life of the process (the graph refers to its work-lists), and its
 * first call must happen outside capture (ROT_ERR_UNSUPPORTED otherwise).
 */
typedef struct { int32_t n_up, n_dn, dim; int64_t offset; } rot_sector;
typedef struct {
    int32_t d;
    const int32_t* site_qn;
    int32_t n_old;
    const rot_sector* old_sec;
    int32_t n_new;
    const rot_sector* new_sec;
    const float* U_blk;
    const int64_t* U_off;
    int32_t n_ops;
    const int32_t* shift;
    const float* O_blk;
    const int64_t* O_off;
    float* out_blk;
    const int64_t* out_off;
} rot_blocked_problem;

ROT_API rot_status rot_batch_blocked(const rot_blocked_problem* p, rot_precision prec,
                             void* workspace, size_t workspace_bytes, void* stream);
ROT_API size_t rot_blocked_workspace_size(const rot_blocked_problem* p);

/*
 * The superblock Hamiltonian applied to a state (Sec. 3.1: Eq. (9) and its
 * quantum-number form Eq. (10)), the product the Davidson iteration of step 2
 * repeats: out = sum over terms of coef * (O_B (x) O_a (x) O_a~ (x) O_B~) psi on
 * [B a a~ B~], H never formed.
 *
 * Blocks B and B~ are given by their (N_up, N_down) sectors (rot_sector, the
 * offset field unused), the sites a and a~ by the d state numbers site_qn
 * (host, d pairs).  The system [B a] has a sector for every Q = q + qn(s); its
 * basis runs over s ascending and, inside, over the states of B sector
 * Q - qn(s).  The environment [a~ B~] likewise: t (the state of a~) ascending,
 * then the states of B~ sector P - qn(t).  psi has definite total numbers
 * `target` and is stored as one dense block per system sector Q whose
 * partner P = target - Q exists: n_Q x r_P, row-major, in ascending
 * (N_up, N_down) order of Q, packed back to back (FP64, device).
 * rot_sb_layout reports the blocks: with arrays of `capacity` entries it
 * writes each block's numbers (qn, 2 per block), rows, cols and element
 * offset; *n_blocks and *total (elements) are always written.
 *
 * Operators of B: n_left_ops, each with a shift (dN_up, dN_down)
 * (left_shift, host, 2 per op) and, per source sector k, the block
 * (q + shift <- q) of dim(q + shift) x dim(q) FP64 values, row-major, at
 * left_blk + left_off[op * n_left + k] (device data; offsets on the host,
 * -1 = absent).  Operators of B~ likewise.  Terms (host): coef; left_op and
 * right_op index those operators (-1 = identity); site_a and site_at are
 * d x d host matrices (row = new state; NULL = identity) whose non-zero
 * entries all change the numbers by one shift.  The four shifts of a term
 * must add to zero.  A term with operators on both B and B~ returns
 * ROT_ERR_UNSUPPORTED (nearest-neighbour chains have none).
 *
 * rot_sb_plan_create checks the problem, builds the work (one list of output
 * tiles, each with the contributions reaching it in term order) and copies it
 * to the device; the operator data must stay valid and unchanged while the
 * plan lives.  rot_sb_apply writes out = H psi (FP64, device, psi's layout,
 * no overlap with psi) on `stream`, allocates nothing (it can be captured in
 * a graph) and is bitwise repeatable.  rot_sb_plan_flops: the multiply-add
 * work of one apply (2 per multiply-add).
 */
typedef struct {
    double coef;
    int32_t left_op, right_op;
    const double* site_a;
    const double* site_at;
} rot_sb_term;
typedef struct {
    int32_t d;
    const int32_t* site_qn;
    int32_t n_left;
    const rot_sector* left;
    int32_t n_right;
    const rot_sector* right;
    int32_t target[2];
    int32_t n_left_ops;
    const int32_t* left_shift;
    const double* left_blk;
    const int64_t* left_off;
    int32_t n_right_ops;
    const int32_t* right_shift;
    const double* right_blk;
    const int64_t* right_off;
    int32_t n_terms;
    const rot_sb_term* terms;
} rot_sb_problem;
typedef struct rot_sb_plan_s* rot_sb_plan;

ROT_API rot_status rot_sb_layout(const rot_sb_problem* p, int32_t capacity, int32_t* n_blocks, int32_t* qn,
                                 int32_t* rows, int32_t* cols, int64_t* offset, int64_t* total);
ROT_API rot_status rot_sb_plan_create(const rot_sb_problem* p, rot_sb_plan* plan);
ROT_API rot_status rot_sb_apply(rot_sb_plan plan, const double* psi, double* out, void* stream);
ROT_API double rot_sb_plan_flops(rot_sb_plan plan);
ROT_API rot_status rot_sb_plan_destroy(rot_sb_plan plan);

/*
 * Sum of two-point expectation values over all pairs of rotated operators,
 * Eq. (11): L = sum_i sum_j <psi| X_i X_j |psi> = sum_ij (X_i^T psi).(X_j psi),
 * reduced in FP64 on the GPU whatever the storage type of X.
 *   X      n_ops matrices mp x mp at X + b*stride_x (float for ROT_FP32 and
 *          ROT_SPLIT_BF16, double for ROT_FP64)
 *   psi    mp doubles (device)
 *   loss   1 double (device), written
 *   pairs  optional n_ops x n_ops doubles (device): <psi|X_i X_j|psi>
 *   grad   optional mp x mp (same type as X, device): dL/dX_k, which is the
 *          same for every k: psi (S psi)^T + (S^T psi) psi^T, S = sum_j X_j
 *   workspace: at least rot_pair_loss_workspace_size(mp, n_ops) bytes
 */
ROT_API rot_status rot_pair_loss(const void* X, int32_t mp, int32_t n_ops, int64_t stride_x,
                         rot_precision prec, const double* psi, double* loss, double* pairs,
                         void* grad, void* workspace, size_t workspace_bytes, void* stream);
ROT_API size_t rot_pair_loss_workspace_size(int32_t mp, int32_t n_ops);

/*
 * Isometry check of a truncation matrix (Sec. 2: the kept eigenvectors are
 * orthonormal; the block basis is complete only up to the truncation):
 * computes max_{a,b} |(U^T U - I)[a,b]| in FP64 on the GPU for a rows x cols
 * row-major U (float or double per prec) with row stride ldu >= cols (0
 * selects cols).  Synchronises `stream`, stores the deviation in
 * *max_dev_host and returns ROT_ERR_NOT_ISOMETRY when it exceeds `tol` or
 * is NaN (a NaN or infinite entry of U makes the deviation NaN or infinite;
 * ROT_OK otherwise).  workspace: at least
 * rot_isometry_workspace_size(rows, cols, prec) bytes, 256-byte aligned.
 */
ROT_API rot_status rot_check_isometry(const void* U, int32_t rows, int32_t cols, int64_t ldu,
                              rot_precision prec, double tol, double* max_dev_host, void* workspace,
                              size_t workspace_bytes, void* stream);
ROT_API size_t rot_isometry_workspace_size(int32_t rows, int32_t cols, rot_precision prec);

/*
 * The system's reduced density matrix and its kept eigenbasis (Sec. 2:
 * Eq. (2), step 4 of the algorithm, Eq. (3)).  The superblock state arrives
 * split by the quantum numbers of the system [B a]: sector k holds psi_k,
 * n x r (FP64, device, row-major, row stride ld_psi >= r), the amplitudes of
 * its n system states with the r environment states of the complementary
 * numbers (r = 0 is allowed; psi may then be NULL).  For every sector the
 * call forms rho_k = psi_k psi_k^T (Eq. (2), real amplitudes) and
 * diagonalises it in FP64 by two-sided block Jacobi, then writes
 *   w  (n doubles, device): the eigenvalues, descending (equal values keep
 *      their order on the diagonal);
 *   V  (n x n doubles, device, row-major, row stride ld_v >= n): column j is
 *      the unit eigenvector of w[j].
 * Then it keeps the m_keep largest eigenvalues over all sectors (equal
 * values: lower sector index first, then earlier position in w) and writes
 *   kept (n_sectors int32, device): states kept per sector; the rotation's
 *      block for sector k is the first kept[k] columns of its V;
 *   eps  (one double, device): the sum of the eigenvalues left out, which is
 *      Eq. (3)'s truncation error 1 - sum(kept w) when psi has unit norm.
 * m_keep >= the total number of states keeps all of them; m_keep >= 0.
 * Convergence: an off-diagonal entry of rho_k counts as zero once
 * |rho_pq| <= 2^-52 tr(rho_k); a sector is done after a full cycle of block
 * pairs without a rotation.  The call synchronises `stream` once per sweep
 * (a 4-byte read) and returns ROT_ERR_NOT_CONVERGED when a sector is still
 * rotating after 80 sweeps (outputs then hold the last iterate).
 * Sizes: 1 <= n <= 4096, r >= 0.  Outputs must not overlap psi or each
 * other.  workspace: rot_density_workspace_size(sectors, n_sectors) bytes,
 * 256-byte aligned.  Returns ROT_OK, ROT_ERR_INVALID_ARG, ROT_ERR_WORKSPACE,
 * ROT_ERR_HIP or ROT_ERR_NOT_CONVERGED.
 */
typedef struct {
    int32_t n, r;
    const double* psi;
    int64_t ld_psi;
    double* w;
    double* V;
    int64_t ld_v;
} rot_dm_sector;

ROT_API size_t rot_density_workspace_size(const rot_dm_sector* sectors, int32_t n_sectors);
ROT_API rot_status rot_density_basis(const rot_dm_sector* sectors, int32_t n_sectors, int64_t m_keep,
                                     int32_t* kept, double* eps, void* workspace, size_t workspace_bytes,
                                     void* stream);

/* Split of float values into bf16 pairs (the split-BF16 operand format):
 * hi[k] = bf16(x[k]), lo[k] = bf16(x[k] - hi[k]), round to nearest even,
 * stored as raw 16-bit patterns.  n elements; device buffers. */
ROT_API rot_status rot_split_bf16(const float* x, int64_t n, uint16_t* hi, uint16_t* lo, void* stream);

/*
 * Per-kernel timing with HIP events recorded on the launch stream around
 * every kernel this library enqueues (measurement support; not in the
 * paper).  rot_profile_enable(1) clears earlier records and starts
 * recording; rot_profile_enable(0) stops.  rot_profile_read waits for the
 * recorded events, writes one line "name launches total_ms\n" per kernel
 * kind into buf (host, len bytes, NUL-terminated, truncated if short),
 * clears the records and returns the number of kernel kinds (or -1 on a
 * HIP error).  Recording is process-wide and mutex-guarded.
 */
ROT_API rot_status rot_profile_enable(int32_t on);
ROT_API int32_t rot_profile_read(char* buf, size_t len);

ROT_API const char* rot_status_string(rot_status s);
ROT_API const char* rot_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
ROT_API int32_t rot_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LIBROT_H */
