/*
 * FP64 CPU oracle for reverse-mode differentiation of CSR sparse-matrix
 * expressions (arXiv 2212.05159).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or helper with the HIP library: every routine below is a
 * plain loop over CSR arrays that follows the definition of the operation
 * it names, in float64, with no blocking, fusion or reordering.  Callers
 * upcast float32 inputs to float64 exactly.
 *
 * Threads: the default build is single-threaded.  A second build of this
 * same file with OpenMP (used only to time the oracle on all host cores)
 * splits the loops over independent rows among threads (the loops marked
 * ROWS_PARALLEL); each row is still computed by one thread in the same
 * order, so both builds return the same bits.  Loops that accumulate into
 * shared entries (the A^T products) stay serial.
 *
 * Conventions: CSR with int32 rowptr[m+1] and colind[nnz] (ascending and
 * unique within a row); dense multi-column operands are row-major with k
 * columns.  Gradient outputs are overwritten.  A NULL gradient pointer
 * skips that gradient.
 *
 * Every function cites the passage of the paper it follows.  "Table 1" is
 * the table of vector-Jacobian products in Section 3; the mask convention
 * (gradients of a sparse input live on that input's stored entries) is the
 * opening of Section 3.1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef int32_t i32;
typedef int64_t i64;

#ifdef _OPENMP
#include <omp.h>
#define ROWS_PARALLEL _Pragma("omp parallel for schedule(static)")
#else
#define ROWS_PARALLEL
#endif

/* Threads the row-parallel loops use (1 in the single-threaded build). */
int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* SpMV, Section 3.1.1; Table 1 (SpMV row).                             */
/* ------------------------------------------------------------------ */

/* y = A x: one inner product per row. */
void or_spmv(i32 m, const i32 *rp, const i32 *ci, const double *v,
             const double *x, double *y)
{
    ROWS_PARALLEL
    for (i32 i = 0; i < m; ++i) {
        double s = 0.0;
        for (i32 e = rp[i]; e < rp[i + 1]; ++e) s += v[e] * x[ci[e]];
        y[i] = s;
    }
}

/* VJP of y = A x with upstream gradient gy (the paper's v):
 *   gx    = A^T gy                      (Table 1, SpMV wrt x)
 *   gvals = (gy x^T) masked to pat(A)   (Table 1, SpMV wrt A)        */
void or_spmv_bwd(i32 m, i32 n, const i32 *rp, const i32 *ci, const double *v,
                 const double *x, const double *gy, double *gx, double *gv)
{
    if (gx) {
        for (i32 j = 0; j < n; ++j) gx[j] = 0.0;
        for (i32 i = 0; i < m; ++i)
            for (i32 e = rp[i]; e < rp[i + 1]; ++e) gx[ci[e]] += v[e] * gy[i];
    }
    if (gv) {
        ROWS_PARALLEL
        for (i32 i = 0; i < m; ++i)
            for (i32 e = rp[i]; e < rp[i + 1]; ++e) gv[e] = gy[i] * x[ci[e]];
    }
}

/* ------------------------------------------------------------------ */
/* SpDMM (sparse times dense), Section 3.1.3; Table 1 (SpDMM row).      */
/* ------------------------------------------------------------------ */

/* C = A B with B (n x k) and C (m x k) dense, row-major. */
void or_spmm(i32 m, i32 k, const i32 *rp, const i32 *ci, const double *v,
             const double *B, double *C)
{
    ROWS_PARALLEL
    for (i32 i = 0; i < m; ++i)
        for (i32 c = 0; c < k; ++c) {
            double s = 0.0;
            for (i32 e = rp[i]; e < rp[i + 1]; ++e)
                s += v[e] * B[(i64)ci[e] * k + c];
            C[(i64)i * k + c] = s;
        }
}

/* VJP of C = A B with upstream gradient G (the paper's V):
 *   gB    = A^T G                    (Table 1, SpDMM wrt B)
 *   gvals = (G B^T) masked to pat(A) (Table 1, SpDMM wrt A)           */
void or_spmm_bwd(i32 m, i32 n, i32 k, const i32 *rp, const i32 *ci,
                 const double *v, const double *B, const double *G,
                 double *gB, double *gv)
{
    if (gB) {
        for (i64 t = 0; t < (i64)n * k; ++t) gB[t] = 0.0;
        for (i32 i = 0; i < m; ++i)
            for (i32 e = rp[i]; e < rp[i + 1]; ++e)
                for (i32 c = 0; c < k; ++c)
                    gB[(i64)ci[e] * k + c] += v[e] * G[(i64)i * k + c];
    }
    if (gv) {
        ROWS_PARALLEL
        for (i32 i = 0; i < m; ++i)
            for (i32 e = rp[i]; e < rp[i + 1]; ++e) {
                double s = 0.0;
                for (i32 c = 0; c < k; ++c)
                    s += G[(i64)i * k + c] * B[(i64)ci[e] * k + c];
                gv[e] = s;
            }
    }
}

/* ------------------------------------------------------------------ */
/* Sparse transpose (Section 3.1.3: the SpDMM backward takes the sparse  */
/* transpose of A).  Counting sort by column, rows ascending within a   */
/* column; perm[t] is the position in A of the t-th entry of A^T.       */
/* ------------------------------------------------------------------ */
void or_transpose(i32 m, i32 n, const i32 *rp, const i32 *ci, i32 *rpT,
                  i32 *ciT, i32 *perm)
{
    for (i32 j = 0; j <= n; ++j) rpT[j] = 0;
    for (i32 e = 0; e < rp[m]; ++e) rpT[ci[e] + 1] += 1;
    for (i32 j = 0; j < n; ++j) rpT[j + 1] += rpT[j];
    i32 *next = (i32 *)malloc(sizeof(i32) * (size_t)(n > 0 ? n : 1));
    for (i32 j = 0; j < n; ++j) next[j] = rpT[j];
    for (i32 i = 0; i < m; ++i)
        for (i32 e = rp[i]; e < rp[i + 1]; ++e) {
            i32 t = next[ci[e]]++;
            ciT[t] = i;
            perm[t] = e;
        }
    free(next);
}

/* ------------------------------------------------------------------ */
/* SpSpMM (sparse times sparse), Section 3.1.2; Table 1 (SpSpMM row);   */
/* gradient flow of Fig. 2.                                            */
/* Pattern is structural: (i,j) is stored when some k has (i,k) in A   */
/* and (k,j) in B, even if the sum is numerically zero.                */
/* ------------------------------------------------------------------ */

/* Row counts of C = A B (A m x n, B n x p).  Writes rpC[m+1] and returns
 * nnz(C), or -1 on allocation failure. */
i64 or_spgemm_rowptr(i32 m, i32 p, const i32 *rpA, const i32 *ciA,
                     const i32 *rpB, const i32 *ciB, i32 *rpC)
{
    i32 *mark = (i32 *)malloc(sizeof(i32) * (size_t)(p > 0 ? p : 1));
    if (!mark) return -1;
    for (i32 j = 0; j < p; ++j) mark[j] = -1;
    i64 total = 0;
    rpC[0] = 0;
    for (i32 i = 0; i < m; ++i) {
        i32 cnt = 0;
        for (i32 a = rpA[i]; a < rpA[i + 1]; ++a) {
            i32 k = ciA[a];
            for (i32 b = rpB[k]; b < rpB[k + 1]; ++b)
                if (mark[ciB[b]] != i) { mark[ciB[b]] = i; ++cnt; }
        }
        total += cnt;
        rpC[i + 1] = (i32)total;
    }
    free(mark);
    return total;
}

static int cmp_i32(const void *a, const void *b)
{
    i32 x = *(const i32 *)a, y = *(const i32 *)b;
    return (x > y) - (x < y);
}

/* Column indices (ascending) and values of C = A B, given rpC.
 * C_ij = sum over k ascending of A_ik B_kj.  Returns 0, or -1 on
 * allocation failure. */
int or_spgemm_fill(i32 m, i32 p, const i32 *rpA, const i32 *ciA,
                   const double *vA, const i32 *rpB, const i32 *ciB,
                   const double *vB, const i32 *rpC, i32 *ciC, double *vC)
{
    i32 *mark = (i32 *)malloc(sizeof(i32) * (size_t)(p > 0 ? p : 1));
    double *acc = (double *)malloc(sizeof(double) * (size_t)(p > 0 ? p : 1));
    if (!mark || !acc) { free(mark); free(acc); return -1; }
    for (i32 j = 0; j < p; ++j) { mark[j] = -1; acc[j] = 0.0; }
    for (i32 i = 0; i < m; ++i) {
        i32 cnt = 0;
        i32 *cols = ciC + rpC[i];
        for (i32 a = rpA[i]; a < rpA[i + 1]; ++a) {
            i32 k = ciA[a];
            for (i32 b = rpB[k]; b < rpB[k + 1]; ++b) {
                i32 j = ciB[b];
                if (mark[j] != i) { mark[j] = i; acc[j] = 0.0; cols[cnt++] = j; }
                acc[j] += vA[a] * vB[b];
            }
        }
        qsort(cols, (size_t)cnt, sizeof(i32), cmp_i32);
        for (i32 t = 0; t < cnt; ++t) vC[rpC[i] + t] = acc[cols[t]];
    }
    free(mark);
    free(acc);
    return 0;
}

/* VJP of C = A B with upstream gradient V stored on pat(C) (gC):
 *   gA = (V B^T) masked to pat(A):  gA[(i,k)] = sum_j V_ij B_kj
 *   gB = (A^T V) masked to pat(B):  gB[(k,j)] = sum_i A_ik V_ij
 * (Table 1, SpSpMM rows; Section 3.1.2).  V_ij is zero off pat(C).
 * Returns 0, or -1 on allocation failure. */
int or_spgemm_bwd(i32 m, i32 n, i32 p, const i32 *rpA, const i32 *ciA,
                  const double *vA, const i32 *rpB, const i32 *ciB,
                  const double *vB, const i32 *rpC, const i32 *ciC,
                  const double *gC, double *gA, double *gB)
{
    (void)n;
    double *vrow = (double *)malloc(sizeof(double) * (size_t)(p > 0 ? p : 1));
    if (!vrow) return -1;
    for (i32 j = 0; j < p; ++j) vrow[j] = 0.0;
    if (gB)
        for (i32 b = 0; b < rpB[n]; ++b) gB[b] = 0.0;
    for (i32 i = 0; i < m; ++i) {
        for (i32 c = rpC[i]; c < rpC[i + 1]; ++c) vrow[ciC[c]] = gC[c];
        for (i32 a = rpA[i]; a < rpA[i + 1]; ++a) {
            i32 k = ciA[a];
            double s = 0.0;
            for (i32 b = rpB[k]; b < rpB[k + 1]; ++b) {
                s += vrow[ciB[b]] * vB[b];
                if (gB) gB[b] += vA[a] * vrow[ciB[b]];
            }
            if (gA) gA[a] = s;
        }
        for (i32 c = rpC[i]; c < rpC[i + 1]; ++c) vrow[ciC[c]] = 0.0;
    }
    free(vrow);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Sparse + sparse, Section 3.1.4; Table 1 (Sp + Sp row).              */
/* C = alpha A + beta B for A, B of the same shape.  The pattern of C  */
/* is the union of the two input patterns, kept structurally: (i,j) is */
/* stored when A or B stores it, even where the sum is zero.           */
/* ------------------------------------------------------------------ */

/* Row counts of the union pattern (A and B both m x n).  Writes
 * rpC[m+1] and returns nnz(C), or -1 on allocation failure. */
i64 or_spadd_rowptr(i32 m, i32 n, const i32 *rpA, const i32 *ciA,
                    const i32 *rpB, const i32 *ciB, i32 *rpC)
{
    i32 *mark = (i32 *)malloc(sizeof(i32) * (size_t)(n > 0 ? n : 1));
    if (!mark) return -1;
    for (i32 j = 0; j < n; ++j) mark[j] = -1;
    i64 total = 0;
    rpC[0] = 0;
    for (i32 i = 0; i < m; ++i) {
        i32 cnt = 0;
        for (i32 a = rpA[i]; a < rpA[i + 1]; ++a)
            if (mark[ciA[a]] != i) { mark[ciA[a]] = i; ++cnt; }
        for (i32 b = rpB[i]; b < rpB[i + 1]; ++b)
            if (mark[ciB[b]] != i) { mark[ciB[b]] = i; ++cnt; }
        total += cnt;
        rpC[i + 1] = (i32)total;
    }
    free(mark);
    return total;
}

/* Column indices (ascending) and values of C = alpha A + beta B, given
 * rpC: C_ij = alpha A_ij + beta B_ij, a term being absent where its
 * input stores no (i,j).  Returns 0, or -1 on allocation failure. */
int or_spadd_fill(i32 m, i32 n, const i32 *rpA, const i32 *ciA,
                  const double *vA, const i32 *rpB, const i32 *ciB,
                  const double *vB, double alpha, double beta,
                  const i32 *rpC, i32 *ciC, double *vC)
{
    i32 *mark = (i32 *)malloc(sizeof(i32) * (size_t)(n > 0 ? n : 1));
    double *acc = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!mark || !acc) { free(mark); free(acc); return -1; }
    for (i32 j = 0; j < n; ++j) { mark[j] = -1; acc[j] = 0.0; }
    for (i32 i = 0; i < m; ++i) {
        i32 cnt = 0;
        i32 *cols = ciC + rpC[i];
        for (i32 a = rpA[i]; a < rpA[i + 1]; ++a) {
            i32 j = ciA[a];
            if (mark[j] != i) { mark[j] = i; acc[j] = 0.0; cols[cnt++] = j; }
            acc[j] += alpha * vA[a];
        }
        for (i32 b = rpB[i]; b < rpB[i + 1]; ++b) {
            i32 j = ciB[b];
            if (mark[j] != i) { mark[j] = i; acc[j] = 0.0; cols[cnt++] = j; }
            acc[j] += beta * vB[b];
        }
        qsort(cols, (size_t)cnt, sizeof(i32), cmp_i32);
        for (i32 t = 0; t < cnt; ++t) vC[rpC[i] + t] = acc[cols[t]];
    }
    free(mark);
    free(acc);
    return 0;
}

/* VJP of C = alpha A + beta B with upstream gradient V stored on pat(C)
 * (gC):  gA = alpha V masked to pat(A),  gB = beta V masked to pat(B)
 * (Table 1, Sp + Sp rows; Section 3.1.4).  Both masks lie inside pat(C).
 * Returns 0, or -1 on allocation failure. */
int or_spadd_bwd(i32 m, i32 n, const i32 *rpA, const i32 *ciA,
                 const i32 *rpB, const i32 *ciB, const i32 *rpC,
                 const i32 *ciC, const double *gC, double alpha, double beta,
                 double *gA, double *gB)
{
    double *vrow = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!vrow) return -1;
    for (i32 j = 0; j < n; ++j) vrow[j] = 0.0;
    for (i32 i = 0; i < m; ++i) {
        for (i32 c = rpC[i]; c < rpC[i + 1]; ++c) vrow[ciC[c]] = gC[c];
        if (gA)
            for (i32 a = rpA[i]; a < rpA[i + 1]; ++a) gA[a] = alpha * vrow[ciA[a]];
        if (gB)
            for (i32 b = rpB[i]; b < rpB[i + 1]; ++b) gB[b] = beta * vrow[ciB[b]];
        for (i32 c = rpC[i]; c < rpC[i + 1]; ++c) vrow[ciC[c]] = 0.0;
    }
    free(vrow);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Level sets of a triangular matrix: the dependency DAG of the         */
/* triangular solve of Section 3.1.5.  For a lower matrix, a row with  */
/* no stored entry left of the diagonal is on level 0, otherwise it is */
/* one above the highest level among the rows it reads.  For an upper  */
/* matrix the same holds with "right of the diagonal".                 */
/* Rows are grouped by level, ascending within a level.                */
/* Returns the number of levels.                                       */
/* ------------------------------------------------------------------ */
i32 or_levels(i32 n, const i32 *rp, const i32 *ci, int lower,
              i32 *level_of_row, i32 *level_ptr, i32 *level_rows)
{
    i32 nlev = 0;
    for (i32 s = 0; s < n; ++s) {
        i32 i = lower ? s : n - 1 - s;
        i32 lv = 0;
        for (i32 e = rp[i]; e < rp[i + 1]; ++e) {
            i32 j = ci[e];
            int dep = lower ? (j < i) : (j > i);
            if (dep && level_of_row[j] + 1 > lv) lv = level_of_row[j] + 1;
        }
        level_of_row[i] = lv;
        if (lv + 1 > nlev) nlev = lv + 1;
    }
    for (i32 l = 0; l <= nlev; ++l) level_ptr[l] = 0;
    for (i32 i = 0; i < n; ++i) level_ptr[level_of_row[i] + 1] += 1;
    for (i32 l = 0; l < nlev; ++l) level_ptr[l + 1] += level_ptr[l];
    i32 *next = (i32 *)malloc(sizeof(i32) * (size_t)(nlev > 0 ? nlev : 1));
    for (i32 l = 0; l < nlev; ++l) next[l] = level_ptr[l];
    for (i32 i = 0; i < n; ++i) level_rows[next[level_of_row[i]]++] = i;
    free(next);
    return nlev;
}

/* ------------------------------------------------------------------ */
/* Sparse triangular solve, Section 3.1.5; Table 1 (SpSolve row).       */
/* ------------------------------------------------------------------ */

/* Solve T x = b for lower (forward substitution) or upper (back
 * substitution) triangular T with a stored, non-unit diagonal.
 * Returns 0, or 1 + the first row whose diagonal is not stored. */
i32 or_trisolve(i32 n, const i32 *rp, const i32 *ci, const double *v,
                int lower, const double *b, double *x)
{
    for (i32 s = 0; s < n; ++s) {
        i32 i = lower ? s : n - 1 - s;
        double acc = b[i], d = 0.0;
        int have_d = 0;
        for (i32 e = rp[i]; e < rp[i + 1]; ++e) {
            i32 j = ci[e];
            if (j == i) { d = v[e]; have_d = 1; }
            else acc -= v[e] * x[j];
        }
        if (!have_d) return i + 1;
        x[i] = acc / d;
    }
    return 0;
}

/* VJP of x = T^{-1} b with upstream gradient gx (the paper's v):
 *   w  = T^{-T} gx                         (Table 1, SpSolve wrt b)
 *   gb = w
 *   gvals[(i,j)] = -w_i x_j on pat(T)      (Table 1, SpSolve wrt A)
 * T^T w = gx is solved column-by-column on T's own rows.
 * Returns 0, or 1 + the first row whose diagonal is not stored. */
i32 or_trisolve_bwd(i32 n, const i32 *rp, const i32 *ci, const double *v,
                    int lower, const double *x, const double *gx, double *gb,
                    double *gv)
{
    double *w = gb;
    for (i32 i = 0; i < n; ++i) w[i] = gx[i];
    /* T^T is upper when T is lower: rows of T are finished from the last
     * one back, each finished w_i is then removed from the rows it feeds. */
    for (i32 s = 0; s < n; ++s) {
        i32 i = lower ? n - 1 - s : s;
        double d = 0.0;
        int have_d = 0;
        for (i32 e = rp[i]; e < rp[i + 1]; ++e)
            if (ci[e] == i) { d = v[e]; have_d = 1; }
        if (!have_d) return i + 1;
        w[i] = w[i] / d;
        for (i32 e = rp[i]; e < rp[i + 1]; ++e)
            if (ci[e] != i) w[ci[e]] -= v[e] * w[i];
    }
    if (gv)
        for (i32 i = 0; i < n; ++i)
            for (i32 e = rp[i]; e < rp[i + 1]; ++e) gv[e] = -w[i] * x[ci[e]];
    return 0;
}

/* ------------------------------------------------------------------ */
/* Conjugate gradient (Section 4.3; Saad) and its reverse mode.         */
/* x0 = 0, r0 = b, p0 = r0.  Step t: q = A p, sigma = p.q,              */
/* alpha = rho/sigma, x += alpha p, r -= alpha q, rho' = r.r,           */
/* beta = rho'/rho, p = r + beta p.  Once rho reaches exactly zero the  */
/* iteration has converged and later steps leave x, r, p unchanged     */
/* (alpha = beta = 0), so no 0/0 arises.                               */
/* ------------------------------------------------------------------ */

static double dot(i32 n, const double *a, const double *b)
{
    double s = 0.0;
    for (i32 i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Runs K steps.  x (out, n).  If R != NULL it receives the residuals
 * r_1..r_K (K x n).  If P, Q, S != NULL they receive p_0..p_{K-1},
 * q_0..q_{K-1} (K x n each) and per-step scalars S[5t..5t+4] =
 * (rho_t, sigma_t, alpha_t, rho_{t+1}, beta_t).  Returns 0. */
int or_cg(i32 n, const i32 *rp, const i32 *ci, const double *v,
          const double *b, i32 K, double *x, double *R, double *P,
          double *Q, double *S)
{
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    for (i32 i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; p[i] = b[i]; }
    double rho = dot(n, r, r);
    for (i32 t = 0; t < K; ++t) {
        or_spmv(n, rp, ci, v, p, q);
        double sigma = dot(n, p, q);
        double alpha = rho != 0.0 ? rho / sigma : 0.0;
        if (P) memcpy(P + (i64)t * n, p, sizeof(double) * (size_t)n);
        if (Q) memcpy(Q + (i64)t * n, q, sizeof(double) * (size_t)n);
        for (i32 i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        double rho1 = dot(n, r, r);
        double beta = rho != 0.0 ? rho1 / rho : 0.0;
        for (i32 i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        if (R) memcpy(R + (i64)t * n, r, sizeof(double) * (size_t)n);
        if (S) {
            S[5 * t + 0] = rho; S[5 * t + 1] = sigma; S[5 * t + 2] = alpha;
            S[5 * t + 3] = rho1; S[5 * t + 4] = beta;
        }
        rho = rho1;
    }
    free(r); free(p); free(q);
    return 0;
}

/* Reverse mode of or_cg.  Upstream gradients: gx (wrt x_K, may be NULL)
 * and gR (wrt r_1..r_K, K x n, may be NULL).  Outputs gv (wrt the values
 * of A on its pattern, not symmetrised) and gb (wrt b).  Each step is
 * undone in reverse order of its statements; the step's q = A p gives
 * gv[(i,j)] += qbar_i p_j and pbar += A^T qbar.  Returns 0. */
int or_cg_bwd(i32 n, const i32 *rp, const i32 *ci, const double *v,
              const double *b, i32 K, const double *gx, const double *gR,
              double *gv, double *gb)
{
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double *R = (double *)malloc(sizeof(double) * (size_t)K * n + 8);
    double *P = (double *)malloc(sizeof(double) * (size_t)K * n + 8);
    double *Q = (double *)malloc(sizeof(double) * (size_t)K * n + 8);
    double *S = (double *)malloc(sizeof(double) * (size_t)K * 5 + 8);
    or_cg(n, rp, ci, v, b, K, x, R, P, Q, S);

    double *xb = (double *)calloc((size_t)n, sizeof(double));
    double *rb = (double *)calloc((size_t)n, sizeof(double));
    double *pb = (double *)calloc((size_t)n, sizeof(double));
    double *qb = (double *)calloc((size_t)n, sizeof(double));
    double *tmp = (double *)calloc((size_t)n, sizeof(double));
    double rhob = 0.0; /* adjoint of rho_{t+1} carried into step t */
    if (gx) for (i32 i = 0; i < n; ++i) xb[i] = gx[i];
    for (i32 e = 0; e < rp[n]; ++e) gv[e] = 0.0;

    for (i32 t = K - 1; t >= 0; --t) {
        const double *p = P + (i64)t * n, *q = Q + (i64)t * n;
        const double *r1 = R + (i64)t * n;            /* r_{t+1} */
        double rho = S[5 * t], sigma = S[5 * t + 1], alpha = S[5 * t + 2];
        double rho1 = S[5 * t + 3], beta = S[5 * t + 4];
        /* upstream gradient on r_{t+1} */
        if (gR) for (i32 i = 0; i < n; ++i) rb[i] += gR[(i64)t * n + i];
        /* p_{t+1} = r_{t+1} + beta p_t */
        double betab = dot(n, pb, p);
        for (i32 i = 0; i < n; ++i) rb[i] += pb[i];
        for (i32 i = 0; i < n; ++i) pb[i] *= beta;
        /* beta = rho_{t+1} / rho_t  (zero once converged) */
        double rhob_t = 0.0;
        if (rho != 0.0) { rhob += betab / rho; rhob_t -= betab * rho1 / (rho * rho); }
        /* rho_{t+1} = r_{t+1} . r_{t+1} */
        for (i32 i = 0; i < n; ++i) rb[i] += 2.0 * rhob * r1[i];
        /* r_{t+1} = r_t - alpha q_t ; x_{t+1} = x_t + alpha p_t */
        double alphab = -dot(n, rb, q) + dot(n, xb, p);
        for (i32 i = 0; i < n; ++i) { qb[i] = -alpha * rb[i]; pb[i] += alpha * xb[i]; }
        /* alpha = rho_t / sigma_t  (zero once converged) */
        double sigmab = 0.0;
        if (rho != 0.0) { rhob_t += alphab / sigma; sigmab = -alphab * rho / (sigma * sigma); }
        /* sigma = p . q */
        for (i32 i = 0; i < n; ++i) { pb[i] += sigmab * q[i]; qb[i] += sigmab * p[i]; }
        /* q = A p */
        or_spmv_bwd(n, n, rp, ci, v, p, qb, tmp, NULL);
        for (i32 i = 0; i < n; ++i) pb[i] += tmp[i];
        for (i32 i = 0; i < n; ++i)
            for (i32 e = rp[i]; e < rp[i + 1]; ++e) gv[e] += qb[i] * p[ci[e]];
        rhob = rhob_t;
    }
    /* rho_0 = r_0 . r_0 ; p_0 = r_0 ; r_0 = b */
    for (i32 i = 0; i < n; ++i) gb[i] = rb[i] + pb[i] + 2.0 * rhob * b[i];

    free(x); free(R); free(P); free(Q); free(S);
    free(xb); free(rb); free(pb); free(qb); free(tmp);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Preconditioned CG (Section 4.3; Saad).  z = M^{-1} r, rho = r.z,     */
/* p = z + beta p.  The preconditioner is either Jacobi (mode 0:        */
/* z = r / diag(A)) or a lower factor L with M = L L^T (mode 1:         */
/* z = L^{-T} (L^{-1} r), two triangular solves), or none (mode 2), or  */
/* the approximate-inverse form of Section 4.3 (mode 3): M = L L^T      */
/* approximates A^{-1} itself and is applied as z = L (L^T r), two      */
/* sparse products.                                                     */
/* Iterates until ||r|| / ||b|| <= tol or maxit; returns the iteration  */
/* count, or -1 on breakdown (non-finite or non-positive curvature).    */
/* hist (maxit+1, may be NULL) receives ||r_t||/||b||.                  */
/* ------------------------------------------------------------------ */
static void apply_prec(i32 n, const i32 *rp, const i32 *ci, const double *v,
                       int mode, const i32 *lrp, const i32 *lci,
                       const double *lv, const double *r, double *z,
                       double *tmp)
{
    if (mode == 0) {
        for (i32 i = 0; i < n; ++i) {
            double d = 0.0;
            for (i32 e = rp[i]; e < rp[i + 1]; ++e) if (ci[e] == i) d = v[e];
            z[i] = r[i] / d;
        }
    } else if (mode == 1) {
        or_trisolve(n, lrp, lci, lv, 1, r, tmp);
        /* L^T z = tmp: the adjoint solve of or_trisolve_bwd gives T^{-T} */
        or_trisolve_bwd(n, lrp, lci, lv, 1, tmp, tmp, z, NULL);
    } else if (mode == 3) {
        /* tmp = L^T r is the input gradient of the SpMV y = L x */
        or_spmv_bwd(n, n, lrp, lci, lv, r, r, tmp, NULL);
        or_spmv(n, lrp, lci, lv, tmp, z);
    } else {
        for (i32 i = 0; i < n; ++i) z[i] = r[i];
    }
}

i32 or_pcg(i32 n, const i32 *rp, const i32 *ci, const double *v,
           const double *b, int mode, const i32 *lrp, const i32 *lci,
           const double *lv, double tol, i32 maxit, double *x, double *hist)
{
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
    if (n <= 0) { free(r); free(z); free(p); free(q); free(tmp); return 0; }
    for (i32 i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; }
    double bn = sqrt(dot(n, b, b));
    apply_prec(n, rp, ci, v, mode, lrp, lci, lv, r, z, tmp);
    for (i32 i = 0; i < n; ++i) p[i] = z[i];
    double rho = dot(n, r, z);
    double rel = bn > 0 ? sqrt(dot(n, r, r)) / bn : 0.0;
    if (hist) hist[0] = rel;
    i32 it = 0, status = 0;
    while (rel > tol && it < maxit) {
        or_spmv(n, rp, ci, v, p, q);
        double sigma = dot(n, p, q);
        if (!(sigma > 0.0) || !isfinite(sigma) || !isfinite(rho)) { status = -1; break; }
        double alpha = rho / sigma;
        for (i32 i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        apply_prec(n, rp, ci, v, mode, lrp, lci, lv, r, z, tmp);
        double rho1 = dot(n, r, z);
        double beta = rho1 / rho;
        for (i32 i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rho = rho1;
        ++it;
        rel = sqrt(dot(n, r, r)) / bn;
        if (hist) hist[it] = rel;
        if (!isfinite(rel)) { status = -1; break; }
    }
    free(r); free(z); free(p); free(q); free(tmp);
    return status < 0 ? -1 : it;
}

/* ------------------------------------------------------------------ */
/* Incomplete Cholesky IC(0) on the lower pattern of a symmetric A       */
/* (Saad, Section 10.3): L_ij for stored (i,j), j < i:                  */
/*   L_ij = (A_ij - sum_{k<j} L_ik L_jk) / L_jj                          */
/*   L_ii = sqrt(A_ii - sum_{k<i} L_ik^2)                                */
/* where the sums run over k stored in both rows of L.  lrp/lci give     */
/* the lower pattern (diagonal last in each row); lv receives values.   */
/* Returns 0, or 1 + the first row with a non-positive pivot.           */
/* ------------------------------------------------------------------ */
i32 or_ic0(i32 n, const i32 *rp, const i32 *ci, const double *v,
           const i32 *lrp, const i32 *lci, double *lv)
{
    for (i32 i = 0; i < n; ++i) {
        for (i32 e = lrp[i]; e < lrp[i + 1]; ++e) {
            i32 j = lci[e];
            double a = 0.0;
            for (i32 f = rp[i]; f < rp[i + 1]; ++f) if (ci[f] == j) a = v[f];
            double s = 0.0;
            /* sparse dot over k < j of rows i and j of L */
            i32 pi = lrp[i], pj = lrp[j];
            while (pi < e && pj < lrp[j + 1] && lci[pj] < j) {
                if (lci[pi] == lci[pj]) { s += lv[pi] * lv[pj]; ++pi; ++pj; }
                else if (lci[pi] < lci[pj]) ++pi;
                else ++pj;
            }
            if (j == i) {
                double d = a - s;
                if (!(d > 0.0)) return i + 1;
                lv[e] = sqrt(d);
            } else {
                lv[e] = (a - s) / lv[lrp[j + 1] - 1];
            }
        }
    }
    return 0;
}

/* The residual-history loss of Section 4.3:
 *   l = sum_{i=1..Nit} w_i ||r_i|| / ||b||,
 *   w_i = gamma^(Nit-i) / sum_{j=1..Nit} gamma^(Nit-j).
 * rnorm holds ||r_1||..||r_Nit||.  Also writes the weights. */
double or_paper_loss(i32 nit, double gamma, const double *rnorm, double bnorm,
                     double *w)
{
    double den = 0.0;
    for (i32 j = 1; j <= nit; ++j) den += pow(gamma, nit - j);
    double l = 0.0;
    for (i32 i = 1; i <= nit; ++i) {
        w[i - 1] = pow(gamma, nit - i) / den;
        l += w[i - 1] * rnorm[i - 1] / bnorm;
    }
    return l;
}
