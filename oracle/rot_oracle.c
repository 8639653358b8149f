/*
 * Oracle for the operator rotation of the density matrix renormalization
 * group (Rincon, Garcia & Hallberg, "Improved parallelization techniques for
 * the density matrix renormalization group").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, double-precision
 * CPU statement of what the GPU library computes.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header or table with the GPU library.
 *
 * Every routine follows the definition in the paper as literally as possible:
 *  - Sec. 2, step 5 and the paragraph after it: an operator Z living on the
 *    block B is first "blocked" onto the enlarged block [B a] (Z tensored with
 *    the identity of the added site), then rotated and decimated with the
 *    density-matrix eigenvectors: Z_new = R Z_[B a] R^+.
 *  - Sec. 3.2: the product is taken in the order "Z R^+ first, then R(Z R^+)".
 *  - The arithmetic is real (the Hubbard Hamiltonian of Eq. (4) is real), so
 *    R^+ = R^T.  We store U = R^T, an (m*d) x m' matrix whose columns are the
 *    kept eigenvectors, with block-site row index r = i*d + s (old block state
 *    i slow, site state s fast), i.e. Z_[B a] = kron(Z, I_d).
 *
 * No blocking, fusion or reordering beyond the definition: the Kronecker
 * product is materialised explicitly and the two products are plain triple
 * loops with ascending summation index.
 *
 * Work over operators is split with the paper's uniform-matrix distribution
 * (Sec. 3.2): with p workers and L operators, each worker owns floor(L/p)
 * contiguous operators and the first mod(L,p) workers own one more.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Sec. 3.2 (uniform-matrix distribution): contiguous range of worker `rank`
 * out of `p` for `n` items. */
void orc_umd_range(int64_t n, int p, int rank, int64_t* lo, int64_t* hi) {
    int64_t q = n / p, r = n % p;
    int64_t begin = rank * q + (rank < r ? rank : r);
    int64_t len = q + (rank < r ? 1 : 0);
    *lo = begin;
    *hi = begin + len;
}

static int orc_threads(int requested) {
#ifdef _OPENMP
    return requested > 0 ? requested : omp_get_max_threads();
#else
    (void)requested;
    return 1;
#endif
}

/* Blocking step (Sec. 2, paragraph after the step list; Sec. 3.2 task ii):
 * A = kron(O, I_d), A[i*d+s, j*d+t] = O[i,j] * delta(s,t).  A is (m*d)^2. */
static void orc_block(int m, int d, const double* O, double* A) {
    int64_t md = (int64_t)m * d;
    memset(A, 0, sizeof(double) * md * md);
    for (int i = 0; i < m; i++)
        for (int j = 0; j < m; j++)
            for (int s = 0; s < d; s++)
                A[((int64_t)i * d + s) * md + (int64_t)j * d + s] = O[(int64_t)i * m + j];
}

/* C (r x c) = X (r x k) * Y (k x c), all row-major, ascending summation. */
static void orc_matmul(int64_t r, int64_t k, int64_t c, const double* X, const double* Y, double* C) {
    memset(C, 0, sizeof(double) * r * c);
    for (int64_t a = 0; a < r; a++)
        for (int64_t t = 0; t < k; t++) {
            double x = X[a * k + t];
            const double* y = Y + t * c;
            double* o = C + a * c;
            for (int64_t b = 0; b < c; b++) o[b] += x * y[b];
        }
}

/* C (r x c) = X^T * Y with X stored (k x r), Y (k x c); ascending summation. */
static void orc_matmul_tn(int64_t r, int64_t k, int64_t c, const double* X, const double* Y, double* C) {
    memset(C, 0, sizeof(double) * r * c);
    for (int64_t a = 0; a < r; a++)
        for (int64_t t = 0; t < k; t++) {
            double x = X[t * r + a];
            const double* y = Y + t * c;
            double* o = C + a * c;
            for (int64_t b = 0; b < c; b++) o[b] += x * y[b];
        }
}

/* C (r x c) = X * Y^T with X (r x k), Y (c x k); ascending summation. */
static void orc_matmul_nt(int64_t r, int64_t k, int64_t c, const double* X, const double* Y, double* C) {
    for (int64_t a = 0; a < r; a++)
        for (int64_t b = 0; b < c; b++) {
            double acc = 0.0;
            for (int64_t t = 0; t < k; t++) acc += X[a * k + t] * Y[b * k + t];
            C[a * c + b] = acc;
        }
}

/*
 * Dense rotation of a batch of operators sharing one U (Sec. 2 step 5,
 * Sec. 3.2):  out_b = U^T kron(O_b, I_d) U.
 *   U   : (m*d) x mp, row-major
 *   O   : n_ops x m x m, operator b at O + b*m*m
 *   out : n_ops x mp x mp
 * Returns 0, or -1 if a scratch allocation failed.
 */
int orc_rotate(int m, int d, int mp, int n_ops, const double* U, const double* O, double* out,
               int nthreads) {
    int p = orc_threads(nthreads);
    int64_t md = (int64_t)m * d;
    int failed = 0;
#ifdef _OPENMP
#pragma omp parallel num_threads(p) reduction(| : failed)
#endif
    {
        int rank = 0;
#ifdef _OPENMP
        rank = omp_get_thread_num();
#endif
        int64_t lo, hi;
        orc_umd_range(n_ops, p, rank, &lo, &hi);
        double* A = NULL;
        double* T = NULL;
        if (hi > lo) {
            A = (double*)malloc(sizeof(double) * md * md);
            T = (double*)malloc(sizeof(double) * md * mp);
            if (!A || !T) failed = 1;
        }
        for (int64_t b = lo; b < hi && !failed; b++) {
            orc_block(m, d, O + b * (int64_t)m * m, A);                 /* Z_[B a] */
            orc_matmul(md, md, mp, A, U, T);                             /* Z R^+  */
            orc_matmul_tn(mp, md, mp, U, T, out + b * (int64_t)mp * mp); /* R (Z R^+) */
        }
        free(A);
        free(T);
    }
    return failed ? -1 : 0;
}

/* Blocking of an operator together with the added site (Sec. 2 step 3, the
 * blocking Z_[B a] <- Z_[B (+) a] for operators that act on the new site):
 * A = kron(X, S), A[i*d+s, j*d+t] = X[i,j] * S[s,t].  X = I_m gives the new
 * site's own operator I_B (x) Z_a; X = P_B (block fermion parity) gives a
 * fermionic site operator with its Jordan-Wigner string over the block; a
 * block operator X gives the block-site product X (x) Z_a. */
static void orc_block_site(int m, int d, const double* X, const double* S, double* A) {
    int64_t md = (int64_t)m * d;
    for (int i = 0; i < m; i++)
        for (int s = 0; s < d; s++)
            for (int j = 0; j < m; j++)
                for (int t = 0; t < d; t++)
                    A[((int64_t)i * d + s) * md + (int64_t)j * d + t] = X[(int64_t)i * m + j] * S[s * d + t];
}

/*
 * Rotation of operators blocked with a site operator:
 *   out_b = U^T kron(X_b, S) U
 *   U   : (m*d) x mp;  X : n_ops x m x m;  S : d x d (shared by the batch)
 *   out : n_ops x mp x mp
 * Same order as orc_rotate: blocked operator times U first, then U^T times
 * that.  Returns 0, or -1 if a scratch allocation failed.
 */
int orc_rotate_site(int m, int d, int mp, int n_ops, const double* U, const double* X, const double* S,
                    double* out, int nthreads) {
    int p = orc_threads(nthreads);
    int64_t md = (int64_t)m * d;
    int failed = 0;
#ifdef _OPENMP
#pragma omp parallel num_threads(p) reduction(| : failed)
#endif
    {
        int rank = 0;
#ifdef _OPENMP
        rank = omp_get_thread_num();
#endif
        int64_t lo, hi;
        orc_umd_range(n_ops, p, rank, &lo, &hi);
        double* A = NULL;
        double* T = NULL;
        if (hi > lo) {
            A = (double*)malloc(sizeof(double) * md * md);
            T = (double*)malloc(sizeof(double) * md * mp);
            if (!A || !T) failed = 1;
        }
        for (int64_t b = lo; b < hi && !failed; b++) {
            orc_block_site(m, d, X + b * (int64_t)m * m, S, A);
            orc_matmul(md, md, mp, A, U, T);
            orc_matmul_tn(mp, md, mp, U, T, out + b * (int64_t)mp * mp);
        }
        free(A);
        free(T);
    }
    return failed ? -1 : 0;
}

/*
 * Selected entries of one operator blocked with a site operator, each on its
 * own from the definition:
 *   out[alpha,beta] = sum_{i,s,j,t} U[i*d+s,alpha] X[i,j] S[s,t] U[j*d+t,beta].
 * Cost m*m*d*d per entry; used to check full-size results at sampled positions.
 */
void orc_rotate_site_entries(int m, int d, int mp, const double* U, const double* X, const double* S,
                             int n_entries, const int32_t* alpha, const int32_t* beta, double* values) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int e = 0; e < n_entries; e++) {
        const int a = alpha[e], b = beta[e];
        double acc = 0.0;
        for (int i = 0; i < m; i++)
            for (int s = 0; s < d; s++) {
                const double ua = U[((int64_t)i * d + s) * mp + a];
                for (int j = 0; j < m; j++) {
                    const double x = X[(int64_t)i * m + j];
                    for (int t = 0; t < d; t++) acc += ua * x * S[s * d + t] * U[((int64_t)j * d + t) * mp + b];
                }
            }
        values[e] = acc;
    }
}

/*
 * Measurements in the superblock state (Sec. 3.2: <Z_i> = <psi0|Z_i|psi0> and
 * <Z_i Z_j>, with correlations between the two blocks taken as products of
 * operators of each block).  The state of [B a a~ B~] is the matrix psi with
 * rows i*d + s (block B state i, site a state s) and columns s'*mR + j (site
 * a~ state s', block B~ state j); dR is the dimension of a~.
 *   orc_expect_block: e_b = sum psi[i*d+s, y] Z_b[i,i'] psi[i'*d+s, y]
 *                     (Z_b on B, identity elsewhere), summed literally.
 *   orc_expect_cross: c[b,k] = <psi| kron(Z_b, I_d) psi kron(I_dR, W_k)^T>,
 *                     with both Kronecker products materialised.
 */
void orc_expect_block(int m, int d, int64_t ncols, const double* psi, int n_ops, const double* Z, double* e) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int b = 0; b < n_ops; b++) {
        const double* z = Z + (int64_t)b * m * m;
        double acc = 0.0;
        for (int i = 0; i < m; i++)
            for (int s = 0; s < d; s++)
                for (int ip = 0; ip < m; ip++) {
                    const double zv = z[(int64_t)i * m + ip];
                    const double* r1 = psi + ((int64_t)i * d + s) * ncols;
                    const double* r2 = psi + ((int64_t)ip * d + s) * ncols;
                    for (int64_t y = 0; y < ncols; y++) acc += r1[y] * zv * r2[y];
                }
        e[b] = acc;
    }
}

int orc_expect_cross(int m, int d, int mR, int dR, const double* psi, int nL, const double* Z, int nR,
                     const double* W, double* c) {
    const int64_t ml = (int64_t)m * d, mr = (int64_t)dR * mR;
    double* A = (double*)malloc(sizeof(double) * ml * ml);   /* kron(Z_b, I_d) */
    double* B = (double*)malloc(sizeof(double) * mr * mr);   /* kron(I_dR, W_k) */
    double* AP = (double*)malloc(sizeof(double) * ml * mr);  /* A psi */
    double* APB = (double*)malloc(sizeof(double) * ml * mr); /* A psi B^T */
    if (!A || !B || !AP || !APB) {
        free(A); free(B); free(AP); free(APB);
        return -1;
    }
    for (int b = 0; b < nL; b++) {
        const double* z = Z + (int64_t)b * m * m;
        memset(A, 0, sizeof(double) * ml * ml);
        for (int i = 0; i < m; i++)
            for (int j = 0; j < m; j++)
                for (int s = 0; s < d; s++) A[((int64_t)i * d + s) * ml + (int64_t)j * d + s] = z[(int64_t)i * m + j];
        orc_matmul(ml, ml, mr, A, psi, AP);
        for (int k = 0; k < nR; k++) {
            const double* w = W + (int64_t)k * mR * mR;
            memset(B, 0, sizeof(double) * mr * mr);
            for (int s = 0; s < dR; s++)
                for (int i = 0; i < mR; i++)
                    for (int j = 0; j < mR; j++) B[((int64_t)s * mR + i) * mr + (int64_t)s * mR + j] = w[(int64_t)i * mR + j];
            orc_matmul_nt(ml, mr, mr, AP, B, APB);
            double acc = 0.0;
            for (int64_t e = 0; e < ml * mr; e++) acc += psi[e] * APB[e];
            c[(int64_t)b * nR + k] = acc;
        }
    }
    free(A); free(B); free(AP); free(APB);
    return 0;
}

/*
 * Selected entries of one rotated operator, each computed on its own straight
 * from the definition:  out[alpha,beta] = sum_{i,j,s} U[i*d+s,alpha] O[i,j] U[j*d+s,beta].
 * Cost m*m*d per entry; used to check full-size results at sampled positions.
 */
void orc_rotate_entries(int m, int d, int mp, const double* U, const double* O, int n_entries,
                        const int32_t* alpha, const int32_t* beta, double* values) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int e = 0; e < n_entries; e++) {
        int a = alpha[e], c = beta[e];
        double acc = 0.0;
        for (int i = 0; i < m; i++)
            for (int s = 0; s < d; s++) {
                double uia = U[((int64_t)i * d + s) * mp + a];
                double inner = 0.0;
                for (int j = 0; j < m; j++)
                    inner += O[(int64_t)i * m + j] * U[((int64_t)j * d + s) * mp + c];
                acc += uia * inner;
            }
        values[e] = acc;
    }
}

/*
 * Adjoint (reverse-mode derivative) of the rotation; not in the paper, it is
 * the transpose of the linear map O -> U^T kron(O,I) U and of the bilinear
 * dependence on U.
 * Given dOut_b = dL/dout_b (mp x mp):
 *   G_b   = U dOut_b U^T                          ((m*d) x (m*d))
 *   dO_b[i,j] = sum_s G_b[i*d+s, j*d+s]           (the fold over the site)
 *   dU    = sum_b ( A_b U dOut_b^T + A_b^T U dOut_b ),  A_b = kron(O_b, I_d)
 * stride_dout = 0 broadcasts one dOut to every operator.
 * dO and/or dU may be NULL.  Returns 0, or -1 on allocation failure.
 */
int orc_adjoint(int m, int d, int mp, int n_ops, const double* U, const double* O,
                const double* dOut, int64_t stride_dout, double* dO, double* dU, int nthreads) {
    int p = orc_threads(nthreads);
    int64_t md = (int64_t)m * d;
    int failed = 0;
    double* dU_part = NULL;
    if (dU) {
        dU_part = (double*)calloc((size_t)p * md * mp, sizeof(double));
        if (!dU_part) return -1;
    }
#ifdef _OPENMP
#pragma omp parallel num_threads(p) reduction(| : failed)
#endif
    {
        int rank = 0;
#ifdef _OPENMP
        rank = omp_get_thread_num();
#endif
        int64_t lo, hi;
        orc_umd_range(n_ops, p, rank, &lo, &hi);
        double *A = NULL, *P = NULL, *G = NULL, *T = NULL, *W = NULL, *Y = NULL;
        if (hi > lo) {
            A = (double*)malloc(sizeof(double) * md * md);
            P = (double*)malloc(sizeof(double) * md * mp);
            G = (double*)malloc(sizeof(double) * md * md);
            T = (double*)malloc(sizeof(double) * md * mp);
            W = (double*)malloc(sizeof(double) * md * mp);
            Y = (double*)malloc(sizeof(double) * md * mp);
            if (!A || !P || !G || !T || !W || !Y) failed = 1;
        }
        for (int64_t b = lo; b < hi && !failed; b++) {
            const double* g = dOut + b * stride_dout;
            if (dO) {
                orc_matmul(md, mp, mp, U, g, P);   /* U dOut */
                orc_matmul_nt(md, mp, md, P, U, G); /* (U dOut) U^T */
                double* o = dO + b * (int64_t)m * m;
                for (int i = 0; i < m; i++)
                    for (int j = 0; j < m; j++) {
                        double acc = 0.0;
                        for (int s = 0; s < d; s++) acc += G[((int64_t)i * d + s) * md + (int64_t)j * d + s];
                        o[(int64_t)i * m + j] = acc;
                    }
            }
            if (dU) {
                double* acc = dU_part + (int64_t)rank * md * mp;
                orc_block(m, d, O + b * (int64_t)m * m, A);
                orc_matmul(md, md, mp, A, U, T);    /* A U      */
                orc_matmul_nt(md, mp, mp, T, g, W); /* A U dOut^T */
                orc_matmul_tn(md, md, mp, A, U, Y); /* A^T U    */
                orc_matmul(md, mp, mp, Y, g, P);    /* A^T U dOut */
                for (int64_t e = 0; e < md * mp; e++) acc[e] += W[e] + P[e];
            }
        }
        free(A); free(P); free(G); free(T); free(W); free(Y);
    }
    if (dU && !failed) {
        /* fixed order over workers: deterministic */
        memset(dU, 0, sizeof(double) * md * mp);
        for (int r = 0; r < p; r++)
            for (int64_t e = 0; e < md * mp; e++) dU[e] += dU_part[(int64_t)r * md * mp + e];
    }
    free(dU_part);
    return failed ? -1 : 0;
}

/*
 * Sum of two-point expectation values, Eq. (11):
 *   L = sum_i sum_j <psi| X_i X_j |psi> = sum_i sum_j (X_i^T psi) . (X_j psi)
 * for n_ops real mp x mp matrices X (stride mp*mp) and a real vector psi.
 * pairs (optional, n_ops x n_ops) receives <psi|X_i X_j|psi>.
 * grad (optional, mp x mp) receives dL/dX_k, identical for every k:
 *   psi (S psi)^T + (S^T psi) psi^T  with S = sum_j X_j.
 */
double orc_pair_loss(int mp, int n_ops, const double* X, const double* psi, double* pairs, double* grad) {
    double* v = (double*)malloc(sizeof(double) * (size_t)n_ops * mp); /* X_i^T psi */
    double* w = (double*)malloc(sizeof(double) * (size_t)n_ops * mp); /* X_j psi */
    if (!v || !w) { free(v); free(w); return NAN; }
    for (int b = 0; b < n_ops; b++) {
        const double* x = X + (int64_t)b * mp * mp;
        for (int a = 0; a < mp; a++) {
            double acc_w = 0.0, acc_v = 0.0;
            for (int c = 0; c < mp; c++) {
                acc_w += x[(int64_t)a * mp + c] * psi[c];
                acc_v += x[(int64_t)c * mp + a] * psi[c];
            }
            w[(int64_t)b * mp + a] = acc_w;
            v[(int64_t)b * mp + a] = acc_v;
        }
    }
    double L = 0.0;
    for (int i = 0; i < n_ops; i++)
        for (int j = 0; j < n_ops; j++) {
            double dot = 0.0;
            for (int a = 0; a < mp; a++) dot += v[(int64_t)i * mp + a] * w[(int64_t)j * mp + a];
            if (pairs) pairs[(int64_t)i * n_ops + j] = dot;
            L += dot;
        }
    if (grad) {
        for (int a = 0; a < mp; a++)
            for (int c = 0; c < mp; c++) {
                double sw = 0.0, sv = 0.0;
                for (int b = 0; b < n_ops; b++) {
                    sw += w[(int64_t)b * mp + c];
                    sv += v[(int64_t)b * mp + a];
                }
                grad[(int64_t)a * mp + c] = psi[a] * sw + sv * psi[c];
            }
    }
    free(v);
    free(w);
    return L;
}

/* max_{a,b} |(U^T U - I)[a,b]| for a rows x cols U: deviation from an
 * isometry (the kept density-matrix eigenvectors are orthonormal, Sec. 2). */
double orc_isometry_deviation(int64_t rows, int64_t cols, const double* U) {
    double worst = 0.0;
    for (int64_t a = 0; a < cols; a++)
        for (int64_t b = 0; b < cols; b++) {
            double acc = 0.0;
            for (int64_t r = 0; r < rows; r++) acc += U[r * cols + a] * U[r * cols + b];
            double dev = fabs(acc - (a == b ? 1.0 : 0.0));
            /* a NaN entry makes the deviation undefined: keep the NaN */
            if (dev != dev || dev > worst) worst = dev;
            if (worst != worst) return worst;
        }
    return worst;
}
