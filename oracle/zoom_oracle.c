/*
 * zoom_oracle.c -- CPU FP64 reference implementation of Zoom-SVD
 * (Jang, Choi, Jung, Kang: "Zoom-SVD: Fast and Memory Efficient Method for
 * Extracting Key Patterns in an Arbitrary Time Range", arXiv 1805.00754).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the tests, the smoke check and the benchmark's CPU
 * baseline leg may load it; the product path never does.  It shares no code,
 * header, constant or helper with the HIP library.
 *
 * Everything is plain double precision, no vendor BLAS, written for a reader
 * who checks it against the paper:
 *   - zo_svd:            SVD primitive (Sec. 2.1).  Householder QR (m > n),
 *                        then one-sided (Hestenes) Jacobi on the square factor.
 *   - zo_store:          storage phase in batch form (Alg. 1, Def. 1, Def. 2):
 *                        rank-k SVD of every b-row block.
 *   - zo_partial_svd:    Partial-SVD of one block (Alg. 3, Eqs. (5)-(6)).
 *   - zo_query:          query phase (Alg. 2): Partial-SVD of the boundary
 *                        blocks, SVD of the vertically stacked Sigma_i V_i^T
 *                        rows, block-diagonal product of Eq. (9).
 *   - zo_direct:         SVD of the raw rows A[t_s:t_e) (Problem 1), the
 *                        ground truth the method approximates.
 *
 * Conventions (the readings of the paper used here):
 *   - Row-major storage everywhere.  A is t x c, row tau = time tick tau.
 *   - Time ranges are 0-based and half-open, [t_s, t_e), n = t_e - t_s.
 *   - Block i holds rows [i*b, min((i+1)*b, t)); the last block may be short.
 *   - Singular values are sorted in descending order, ties kept in index
 *     order.  A singular value sigma_j <= rank_tol * sigma_1 is numerically
 *     zero: its triplet is zeroed and it does not count in the rank.
 *   - Sign rule: each kept pair (u_j, v_j) is flipped so that the entry of v_j
 *     with the largest magnitude (lowest index on ties) is positive.
 *   - Partial-SVD keeps all numerically non-zero triplets (no truncation
 *     beyond numerical rank), so the stitched result is exact when every
 *     block has rank <= k.
 *   - Energy threshold xi (Eq. (1)), optional: with 0 < xi < 1 every
 *     low-rank approximation of the method (the block SVDs of the storage
 *     phase, the Partial-SVD of a boundary block, the SVD of the stacked
 *     matrix) keeps the smallest rank whose leading squared singular values
 *     reach xi times the sum of all of them, within the other caps (k, k_q,
 *     numerical rank).  xi = 0 (or >= 1) turns the rule off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

#define ZO_MAX_SWEEPS 80

/* --------------------------------------------------------------------------
 * Householder QR of an m x n column-major matrix X (m >= n), in place.
 * On return the upper triangle of X holds R; the Householder vectors are kept
 * in H (m x n column-major, vector j stored in rows j..m-1 of column j).
 * Textbook algorithm (Golub & Van Loan, Alg. 5.2.1).
 * ------------------------------------------------------------------------ */
static void householder_qr(int64_t m, int64_t n, double *X, double *H)
{
    memset(H, 0, sizeof(double) * (size_t)(m * n));
    for (int64_t j = 0; j < n; ++j) {
        double *xj = X + j * m;
        double norm2 = 0.0;
        for (int64_t i = j; i < m; ++i) norm2 += xj[i] * xj[i];
        double norm = sqrt(norm2);
        double *v = H + j * m;
        if (norm == 0.0) continue;                 /* zero column: H_j = I */
        double alpha = (xj[j] >= 0.0) ? -norm : norm;
        for (int64_t i = j; i < m; ++i) v[i] = xj[i];
        v[j] -= alpha;
        double vnorm2 = 0.0;
        for (int64_t i = j; i < m; ++i) vnorm2 += v[i] * v[i];
        double vnorm = sqrt(vnorm2);
        if (vnorm == 0.0) continue;
        for (int64_t i = j; i < m; ++i) v[i] /= vnorm;
        /* apply H_j = I - 2 v v^T to columns j..n-1 */
        for (int64_t q = j; q < n; ++q) {
            double *xq = X + q * m;
            double d = 0.0;
            for (int64_t i = j; i < m; ++i) d += v[i] * xq[i];
            for (int64_t i = j; i < m; ++i) xq[i] -= 2.0 * d * v[i];
        }
    }
}

/* x <- H_0 H_1 ... H_{n-1} x  for a length-m vector x (applies Q of the QR
 * factorisation to a vector that is zero below row n). */
static void householder_apply_q(int64_t m, int64_t n, const double *H, double *x)
{
    for (int64_t j = n - 1; j >= 0; --j) {
        const double *v = H + j * m;
        double d = 0.0;
        for (int64_t i = j; i < m; ++i) d += v[i] * x[i];
        if (d == 0.0) continue;
        for (int64_t i = j; i < m; ++i) x[i] -= 2.0 * d * v[i];
    }
}

/* --------------------------------------------------------------------------
 * One-sided Jacobi (Hestenes) on the columns of W (m x n column-major),
 * accumulating the rotations in V (n x n column-major, starts as I).
 * A pair (p, q) is rotated when |w_p . w_q| > tol * ||w_p|| ||w_q||,
 * tol = sqrt(m) * eps.  The rotation zeroes w_p . w_q exactly in exact
 * arithmetic (Golub & Van Loan Sec. 8.6.3; Demmel & Veselic 1992).
 * A column whose norm is at the rounding level of the whole matrix,
 * ||w|| <= m eps ||W||_F, is numerically zero and is not rotated (otherwise
 * rounding noise in exactly rank-deficient input never settles).
 * Returns the number of sweeps, or -1 if the sweep cap was hit.
 * ------------------------------------------------------------------------ */
static int one_sided_jacobi(int64_t m, int64_t n, double *W, double *V)
{
    const double tol = sqrt((double)m) * DBL_EPSILON;
    double fro2 = 0.0;
    for (int64_t i = 0; i < m * n; ++i) fro2 += W[i] * W[i];
    const double floor2 = ((double)m * DBL_EPSILON) * ((double)m * DBL_EPSILON) * fro2;
    for (int sweep = 1; sweep <= ZO_MAX_SWEEPS; ++sweep) {
        int64_t rotated = 0;
        for (int64_t p = 0; p + 1 < n; ++p) {
            for (int64_t q = p + 1; q < n; ++q) {
                double *wp = W + p * m, *wq = W + q * m;
                double alpha = 0.0, beta = 0.0, gamma = 0.0;
                for (int64_t i = 0; i < m; ++i) {
                    alpha += wp[i] * wp[i];
                    beta += wq[i] * wq[i];
                    gamma += wp[i] * wq[i];
                }
                if (alpha <= floor2 || beta <= floor2) continue;
                if (fabs(gamma) <= tol * sqrt(alpha) * sqrt(beta)) continue;
                double zeta = (beta - alpha) / (2.0 * gamma);
                double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double cs = 1.0 / sqrt(1.0 + t * t);
                double sn = cs * t;
                for (int64_t i = 0; i < m; ++i) {
                    double a = wp[i], bq = wq[i];
                    wp[i] = cs * a - sn * bq;
                    wq[i] = sn * a + cs * bq;
                }
                double *vp = V + p * n, *vq = V + q * n;
                for (int64_t i = 0; i < n; ++i) {
                    double a = vp[i], bq = vq[i];
                    vp[i] = cs * a - sn * bq;
                    vq[i] = sn * a + cs * bq;
                }
                ++rotated;
            }
        }
        if (rotated == 0) return sweep;
    }
    return -1;
}

/* --------------------------------------------------------------------------
 * zo_svd: thin SVD of an m x n row-major matrix A (leading dimension lda).
 * r = min(m, n).  Outputs (row-major):
 *   U  m x r   (ldu >= r),   column j = u_j
 *   s  r       descending
 *   V  n x r   (ldv >= r),   column j = v_j
 * Only the first nvec singular vector pairs are formed (nvec <= r); the
 * other columns of U and V are left zero.  All r singular values are
 * returned.  Triplets with s_j <= rank_tol * s_1 are zeroed; *rank counts
 * the others.  Returns the Jacobi sweep count, or -1 on non-convergence.
 * ------------------------------------------------------------------------ */
int zo_svd(int64_t m, int64_t n, const double *A, int64_t lda, double rank_tol, int64_t nvec,
           double *U, int64_t ldu, double *s, double *V, int64_t ldv, int32_t *rank)
{
    const int transposed = (m < n);
    /* Work on B = A (mm x nn, mm >= nn) or B = A^T. */
    const int64_t mm = transposed ? n : m;
    const int64_t nn = transposed ? m : n;
    const int64_t r = nn;
    if (nvec > r) nvec = r;
    double *B = (double *)malloc(sizeof(double) * (size_t)(mm * nn));   /* col-major */
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double a = A[i * lda + j];
            if (!transposed) B[j * mm + i] = a;          /* B(i,j) = A(i,j) */
            else             B[i * mm + j] = a;          /* B(j,i) = A(i,j) */
        }

    /* Precondition a tall B with Householder QR: B = Q R, Jacobi on R. */
    const int precond = (mm > nn);
    double *W, *Hh = NULL;
    if (precond) {
        Hh = (double *)malloc(sizeof(double) * (size_t)(mm * nn));
        householder_qr(mm, nn, B, Hh);
        W = (double *)calloc((size_t)(nn * nn), sizeof(double));
        for (int64_t j = 0; j < nn; ++j)
            for (int64_t i = 0; i <= j; ++i) W[j * nn + i] = B[j * mm + i];   /* R */
    } else {
        W = B;
        B = NULL;
    }
    const int64_t wm = precond ? nn : mm;                 /* rows of W */
    double *J = (double *)calloc((size_t)(nn * nn), sizeof(double));
    for (int64_t j = 0; j < nn; ++j) J[j * nn + j] = 1.0;
    int sweeps = one_sided_jacobi(wm, nn, W, J);

    /* sigma_j = ||w_j||, sort descending, ties by index (insertion sort). */
    double *sig = (double *)malloc(sizeof(double) * (size_t)nn);
    int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)nn);
    for (int64_t j = 0; j < nn; ++j) {
        double acc = 0.0;
        for (int64_t i = 0; i < wm; ++i) acc += W[j * wm + i] * W[j * wm + i];
        sig[j] = sqrt(acc);
        ord[j] = j;
    }
    for (int64_t a = 1; a < nn; ++a) {
        int64_t key = ord[a];
        int64_t b2 = a - 1;
        while (b2 >= 0 && sig[ord[b2]] < sig[key]) { ord[b2 + 1] = ord[b2]; --b2; }
        ord[b2 + 1] = key;
    }
    const double s1 = nn > 0 ? sig[ord[0]] : 0.0;
    int32_t rk = 0;
    double *left = (double *)malloc(sizeof(double) * (size_t)mm);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t jj = 0; jj < r; ++jj) U[i * ldu + jj] = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t jj = 0; jj < r; ++jj) V[i * ldv + jj] = 0.0;
    for (int64_t jj = 0; jj < r; ++jj) {
        const int64_t j = ord[jj];
        const double sj = sig[j];
        const int keep = (sj > rank_tol * s1) && sj > 0.0;
        s[jj] = keep ? sj : 0.0;
        if (!keep) continue;
        ++rk;
        if (jj >= nvec) continue;
        /* Right vector of B: column j of J.  Left vector of B: w_j / sigma_j,
         * mapped back through Q when preconditioned. */
        const double *vj = J + j * nn;
        const double *wj = W + j * wm;
        for (int64_t i = 0; i < mm; ++i) left[i] = (i < wm) ? wj[i] / sj : 0.0;
        if (precond) householder_apply_q(mm, nn, Hh, left);
        /* For A = B: u = left, v = vj.  For A = B^T: u = vj, v = left. */
        const double *uu = transposed ? vj : left;
        const double *vv = transposed ? left : vj;
        /* sign rule on v */
        int64_t imax = 0;
        double vmax = -1.0;
        for (int64_t i = 0; i < n; ++i)
            if (fabs(vv[i]) > vmax) { vmax = fabs(vv[i]); imax = i; }
        const double flip = (vv[imax] < 0.0) ? -1.0 : 1.0;
        for (int64_t i = 0; i < m; ++i) U[i * ldu + jj] = flip * uu[i];
        for (int64_t i = 0; i < n; ++i) V[i * ldv + jj] = flip * vv[i];
    }
    if (rank) *rank = rk;
    free(left); free(ord); free(sig); free(J);
    free(W); free(Hh); free(B);
    return sweeps;
}

/* --------------------------------------------------------------------------
 * Energy-threshold rank (Eq. (1)).  s holds all r singular values in
 * descending order.  Returns the smallest k' >= 1 with
 *     sum_{j < k'} s_j^2 >= xi * sum_{j < r} s_j^2,
 * or r when xi <= 0 or xi >= 1 (no threshold) or when s is all zero.
 * ------------------------------------------------------------------------ */
int64_t zo_xi_rank(const double *s, int64_t r, double xi)
{
    if (!(xi > 0.0 && xi < 1.0)) return r;
    double total = 0.0;
    for (int64_t j = 0; j < r; ++j) total += s[j] * s[j];
    if (total <= 0.0) return r;
    double run = 0.0;
    for (int64_t j = 0; j < r; ++j) {
        run += s[j] * s[j];
        if (run >= xi * total) return j + 1;
    }
    return r;
}

/* --------------------------------------------------------------------------
 * Block index math (Def. 1 and Alg. 3, read for 0-based half-open ranges).
 * ------------------------------------------------------------------------ */
int64_t zo_num_blocks(int64_t t, int64_t b) { return (t + b - 1) / b; }
int64_t zo_block_rows(int64_t t, int64_t b, int64_t i)
{
    int64_t r = t - i * b;
    return r < b ? r : b;
}

/* S, E: first and last touched block; lo: first kept row inside S; hi: one
 * past the last kept row inside E.  Alg. 3 writes S = t_s/b, b_S = b - t_s%b,
 * E = t_e/b, b_E = t_e%b; with a half-open range, b_E = 0 means block t_e/b
 * contributes nothing, so the last touched block is (t_e-1)/b. */
void zo_query_blocks(int64_t t_s, int64_t t_e, int64_t b, int64_t *S, int64_t *E,
                     int64_t *lo, int64_t *hi)
{
    *S = t_s / b;
    *E = (t_e - 1) / b;
    *lo = t_s - (*S) * b;
    *hi = t_e - (*E) * b;
}

/* --------------------------------------------------------------------------
 * Storage phase, batch form (Alg. 1 / Def. 1 / Def. 2).
 *   A:    t x c row-major (lda)
 *   Uall: t x k row-major; rows of block i hold U_(i) (rows_i x k)
 *   S:    nb x k;  block i holds Sigma_(i) (zero-padded past k_i)
 *   V:    nb x c x k; block i holds V_(i) (c x k, column j = v_j)
 *   kk:   nb;  k_i = min(k, numerical rank of A_(i), xi rank of Eq. (1))
 * Returns the number of blocks whose Jacobi did not converge.
 * ------------------------------------------------------------------------ */
int zo_store(const double *A, int64_t t, int64_t c, int64_t lda, int64_t b, int32_t k,
             double rank_tol, double xi, double *Uall, double *S, double *V, int32_t *kk)
{
    const int64_t nb = zo_num_blocks(t, b);
    int failures = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : failures)
    for (int64_t i = 0; i < nb; ++i) {
        const int64_t rows = zo_block_rows(t, b, i);
        const int64_t r = rows < c ? rows : c;
        double *Ub = (double *)malloc(sizeof(double) * (size_t)(rows * r));
        double *sb = (double *)malloc(sizeof(double) * (size_t)r);
        double *Vb = (double *)malloc(sizeof(double) * (size_t)(c * r));
        int32_t rank = 0;
        int sw = zo_svd(rows, c, A + i * b * lda, lda, rank_tol, k, Ub, r, sb, Vb, r, &rank);
        if (sw < 0) ++failures;
        int32_t ki = rank < k ? rank : k;
        const int64_t kx = zo_xi_rank(sb, r, xi);      /* Eq. (1) over all r values */
        if (kx < ki) ki = (int32_t)kx;
        kk[i] = ki;
        for (int64_t j = 0; j < k; ++j) S[i * k + j] = j < ki ? sb[j] : 0.0;
        for (int64_t row = 0; row < rows; ++row)
            for (int64_t j = 0; j < k; ++j)
                Uall[(i * b + row) * k + j] = j < ki ? Ub[row * r + j] : 0.0;
        for (int64_t row = 0; row < c; ++row)
            for (int64_t j = 0; j < k; ++j)
                V[(i * c + row) * k + j] = j < ki ? Vb[row * r + j] : 0.0;
        free(Ub); free(sb); free(Vb);
    }
    return failures;
}

/* --------------------------------------------------------------------------
 * Partial-SVD of block i restricted to its rows [r0, r1) (Alg. 3, Eqs. 5-6):
 *   P = X U_(i) Sigma_(i)  (the kept rows of U_(i), columns scaled by sigma)
 *   P = U~ Sigma~ V~^T,   U' = U~,  Sigma' = Sigma~,  V' = V_(i) V~
 * m = r1 - r0 rows, rp = min(m, k) triplets, those past the numerical rank
 * and past the xi rank (Eq. (1)) zeroed.  Outputs:
 *   Up: m x rp,  sp: rp,  Vp: c x rp  (row-major).
 * ------------------------------------------------------------------------ */
int zo_partial_svd(const double *Uall, const double *S, const double *V, int64_t c,
                   int64_t b, int32_t k, int64_t i, int64_t r0, int64_t r1, double rank_tol,
                   double xi, double *Up, double *sp, double *Vp, int32_t *rank)
{
    const int64_t m = r1 - r0;
    const int64_t rp = m < k ? m : k;
    double *P = (double *)malloc(sizeof(double) * (size_t)(m * k));
    for (int64_t row = 0; row < m; ++row)
        for (int64_t j = 0; j < k; ++j)
            P[row * k + j] = Uall[(i * b + r0 + row) * k + j] * S[i * k + j];
    double *Vt = (double *)malloc(sizeof(double) * (size_t)(k * rp));   /* V~ : k x rp */
    int sw = zo_svd(m, k, P, k, rank_tol, rp, Up, rp, sp, Vt, rp, rank);
    /* low-rank approximation with threshold xi (Alg. 3, Eq. (1)): the
     * triplets past the xi rank of P's rp singular values are dropped */
    const int64_t kx = zo_xi_rank(sp, rp, xi);
    if (kx < *rank) *rank = (int32_t)kx;
    for (int64_t j = *rank; j < rp; ++j) {
        sp[j] = 0.0;
        for (int64_t row = 0; row < m; ++row) Up[row * rp + j] = 0.0;
        for (int64_t l = 0; l < k; ++l) Vt[l * rp + j] = 0.0;
    }
    /* V' = V_(i) V~  (c x k times k x rp) */
    const double *Vi = V + i * c * k;
    for (int64_t row = 0; row < c; ++row)
        for (int64_t j = 0; j < rp; ++j) {
            double acc = 0.0;
            for (int64_t l = 0; l < k; ++l) acc += Vi[row * k + l] * Vt[l * rp + j];
            Vp[row * rp + j] = acc;
        }
    free(P); free(Vt);
    return sw;
}

/* --------------------------------------------------------------------------
 * Query phase (Alg. 2) for the range [t_s, t_e), truncated to rank kq (and
 * to the xi rank of the stacked matrix, Eq. (1)).
 *   Uo: n x kq,  so: kq,  Vo: c x kq  (row-major); *kout = rank kept
 *   (<= kq).  Columns past *kout are zero.
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t block, r0, r1;   /* block index and the kept rows inside it     */
    int64_t rows_m;          /* rows this block contributes to the stack    */
    double *Ublk;            /* left factor: (r1-r0) x rows_m               */
    int owns;                /* Ublk was allocated by the Partial-SVD        */
} zo_piece;

int zo_query(const double *Uall, const double *S, const double *V, int64_t t, int64_t c,
             int64_t b, int32_t k, int64_t t_s, int64_t t_e, int32_t kq, double rank_tol,
             double xi, double *Uo, double *so, double *Vo, int32_t *kout)
{
    int64_t Sb, Eb, lo, hi;
    zo_query_blocks(t_s, t_e, b, &Sb, &Eb, &lo, &hi);
    const int64_t npieces = Eb - Sb + 1;
    const int64_t n = t_e - t_s;
    zo_piece *pc = (zo_piece *)calloc((size_t)npieces, sizeof(zo_piece));
    /* Stack rows: at most k per piece. */
    double *M = (double *)calloc((size_t)(npieces * k * c), sizeof(double));
    int64_t K = 0;
    int bad = 0;
    for (int64_t p = 0; p < npieces; ++p) {
        const int64_t i = Sb + p;
        const int64_t rows = zo_block_rows(t, b, i);
        const int64_t r0 = (i == Sb) ? lo : 0;
        const int64_t r1 = (i == Eb) ? hi : rows;
        pc[p].block = i; pc[p].r0 = r0; pc[p].r1 = r1;
        const int partial = (r0 != 0) || (r1 != rows);
        if (partial) {
            /* Alg. 3: Partial-SVD of X U_(i) Sigma_(i). */
            const int64_t m = r1 - r0;
            const int64_t rp = m < k ? m : k;
            double *Up = (double *)malloc(sizeof(double) * (size_t)(m * rp));
            double *sp = (double *)malloc(sizeof(double) * (size_t)rp);
            double *Vp = (double *)malloc(sizeof(double) * (size_t)(c * rp));
            int32_t rk;
            if (zo_partial_svd(Uall, S, V, c, b, k, i, r0, r1, rank_tol, xi, Up, sp, Vp, &rk) < 0)
                bad = 1;
            /* Stack rows Sigma' V'^T (rp x c). */
            for (int64_t j = 0; j < rp; ++j)
                for (int64_t col = 0; col < c; ++col)
                    M[(K + j) * c + col] = sp[j] * Vp[col * rp + j];
            pc[p].rows_m = rp;
            pc[p].Ublk = Up;
            pc[p].owns = 1;
            free(sp); free(Vp);
        } else {
            /* Whole block: stored Sigma_(i) V_(i)^T (k x c), U_(i) as is. */
            for (int64_t j = 0; j < k; ++j)
                for (int64_t col = 0; col < c; ++col)
                    M[(K + j) * c + col] = S[i * k + j] * V[(i * c + col) * k + j];
            pc[p].rows_m = k;
            pc[p].Ublk = (double *)(Uall + (i * b) * k);   /* rows x k, ld k */
            pc[p].owns = 0;
        }
        K += pc[p].rows_m;
    }
    /* Alg. 2, the SVD of the stacked matrix (K x c), truncated to k_q. */
    const int64_t r = K < c ? K : c;
    double *Ur = (double *)malloc(sizeof(double) * (size_t)(K * r));
    double *sr = (double *)malloc(sizeof(double) * (size_t)r);
    double *Vr = (double *)malloc(sizeof(double) * (size_t)(c * r));
    int32_t rk = 0;
    if (zo_svd(K, c, M, c, rank_tol, kq, Ur, r, sr, Vr, r, &rk) < 0) bad = 1;
    int32_t ko = rk < kq ? rk : kq;
    const int64_t kx = zo_xi_rank(sr, r, xi);   /* Eq. (1) over all r values of M */
    if (kx < ko) ko = (int32_t)kx;
    *kout = ko;
    for (int64_t j = 0; j < kq; ++j) so[j] = j < ko ? sr[j] : 0.0;
    for (int64_t row = 0; row < c; ++row)
        for (int64_t j = 0; j < kq; ++j) Vo[row * kq + j] = j < ko ? Vr[row * r + j] : 0.0;
    /* Alg. 2, the block-diagonal product, Eq. (9): U = [U'_S U'_r(S); U_(S+1) U_r(S+1); ...].
     * Skipped when the caller asks for Sigma and V only (Uo == NULL). */
    int64_t krow = 0, orow = 0;
    for (int64_t p = 0; p < npieces; ++p) {
        if (!Uo) {
            if (pc[p].owns) free(pc[p].Ublk);
            continue;
        }
        const int64_t m = pc[p].r1 - pc[p].r0;
        const int64_t w = pc[p].rows_m;
        const int64_t off = pc[p].owns ? 0 : pc[p].r0;   /* whole blocks start at r0 = 0 */
        for (int64_t row = 0; row < m; ++row)
            for (int64_t j = 0; j < kq; ++j) {
                double acc = 0.0;
                if (j < ko)
                    for (int64_t l = 0; l < w; ++l)
                        acc += pc[p].Ublk[(off + row) * w + l] * Ur[(krow + l) * r + j];
                Uo[(orow + row) * kq + j] = acc;
            }
        krow += w;
        orow += m;
        if (pc[p].owns) free(pc[p].Ublk);
    }
    (void)n;
    free(Ur); free(sr); free(Vr); free(M); free(pc);
    return bad ? -1 : 0;
}

/* Many queries at once, parallel over queries.  Outputs are concatenated:
 * query q writes U at Uo + uoff[q] (n_q x kq[q]), sigma at so + soff[q],
 * V at Vo + voff[q] (c x kq[q]).  Uo == NULL: Sigma and V only. */
int zo_query_batch(const double *Uall, const double *S, const double *V, int64_t t, int64_t c,
                   int64_t b, int32_t k, int32_t nq, const int64_t *ts, const int64_t *te,
                   const int32_t *kq, double rank_tol, double xi, double *Uo, const int64_t *uoff,
                   double *so, const int64_t *soff, double *Vo, const int64_t *voff,
                   int32_t *kout)
{
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (int32_t q = 0; q < nq; ++q) {
        if (zo_query(Uall, S, V, t, c, b, k, ts[q], te[q], kq[q], rank_tol, xi,
                     Uo ? Uo + uoff[q] : NULL,
                     so + soff[q], Vo + voff[q], kout + q) < 0)
            ++bad;
    }
    return bad;
}

/* --------------------------------------------------------------------------
 * Direct SVD of the raw rows A[t_s:t_e) truncated to kq (Problem 1).
 * ------------------------------------------------------------------------ */
int zo_direct(const double *A, int64_t c, int64_t lda, int64_t t_s, int64_t t_e, int32_t kq,
              double rank_tol, double *Uo, double *so, double *Vo, int32_t *kout)
{
    const int64_t n = t_e - t_s;
    const int64_t r = n < c ? n : c;
    double *U = (double *)malloc(sizeof(double) * (size_t)(n * r));
    double *s = (double *)malloc(sizeof(double) * (size_t)r);
    double *Vv = (double *)malloc(sizeof(double) * (size_t)(c * r));
    int32_t rk = 0;
    int sw = zo_svd(n, c, A + t_s * lda, lda, rank_tol, kq, U, r, s, Vv, r, &rk);
    const int32_t ko = rk < kq ? rk : kq;
    *kout = ko;
    for (int64_t j = 0; j < kq; ++j) so[j] = j < ko ? s[j] : 0.0;
    for (int64_t row = 0; row < n; ++row)
        for (int64_t j = 0; j < kq; ++j) Uo[row * kq + j] = j < ko ? U[row * r + j] : 0.0;
    for (int64_t row = 0; row < c; ++row)
        for (int64_t j = 0; j < kq; ++j) Vo[row * kq + j] = j < ko ? Vv[row * r + j] : 0.0;
    free(U); free(s); free(Vv);
    return sw < 0 ? -1 : 0;
}

/* Many direct SVDs at once (Problem 1 for each range), parallel over ranges;
 * outputs laid out as in zo_query_batch. */
int zo_direct_batch(const double *A, int64_t c, int64_t lda, int32_t nq, const int64_t *ts,
                    const int64_t *te, const int32_t *kq, double rank_tol, double *Uo,
                    const int64_t *uoff, double *so, const int64_t *soff, double *Vo,
                    const int64_t *voff, int32_t *kout)
{
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (int32_t q = 0; q < nq; ++q) {
        if (zo_direct(A, c, lda, ts[q], te[q], kq[q], rank_tol, Uo + uoff[q], so + soff[q],
                      Vo + voff[q], kout + q) < 0)
            ++bad;
    }
    return bad;
}

/* Threads of the parallel loops above (timing of a one-thread baseline). */
void zo_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int zo_max_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
