/*
 * csrad: differentiable CSR sparse-matrix kernels for AMD Instinct MI355X
 * (gfx950), after "Optimized Sparse Matrix Operations for Reverse Mode
 * Automatic Differentiation" (arXiv 2212.05159).
 *
 * Plain C ABI over hand-written HIP kernels.  Every pointer argument is
 * device memory owned by the caller unless its name ends in _host.  The
 * library never allocates or frees memory: calls that need scratch space
 * take a caller-allocated workspace whose size a *_workspace query gives.
 * Every call is asynchronous on `stream` (a hipStream_t passed as void*;
 * NULL is the default stream) except the three that return a count to
 * the host (csr_spgemm_symbolic, csr_spadd_symbolic and
 * csr_trisolve_analyze), which synchronise the stream.  No exception or abort crosses the ABI: each call returns a
 * status code.  Host-side checks are O(1) (null pointers, shapes, dtype);
 * the pattern invariants below are preconditions that only csr_validate
 * checks.
 *
 * Sparse operands are CSR: rowptr[nrows+1], colind[nnz] with column
 * indices ascending and unique within each row, vals[nnz].  Indices are
 * int32.  Values and every dense operand of one call share one type,
 * float32 or float64 (csrad_csr.dtype).  Dense multi-column operands are
 * row-major with a leading dimension (elements between rows) >= k.
 *
 * Gradients follow the sparse-gradient convention of Section 3.1: the
 * gradient with respect to a sparse input is a value array on that
 * input's own pattern (one entry per stored value, stored zeros
 * included).  Gradient outputs are overwritten, not accumulated.  A NULL
 * gradient output skips its kernel.
 */
#ifndef CSRAD_H
#define CSRAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define CSRAD_OK 0
#define CSRAD_EINVAL (-1)     /* null pointer, bad shape, k <= 0, ld < k  */
#define CSRAD_EDTYPE (-2)     /* unsupported or mismatched value type      */
#define CSRAD_EPATTERN (-3)   /* malformed CSR (csr_validate only)         */
#define CSRAD_ESINGULAR (-4)  /* a triangular row has no stored diagonal   */
#define CSRAD_EWORKSPACE (-5) /* workspace missing or too small            */
#define CSRAD_EHIP (-6)       /* HIP launch or runtime error               */
#define CSRAD_EOVERFLOW (-7)  /* a result does not fit int32 indexing      */

/* Value types. */
#define CSRAD_F32 0
#define CSRAD_F64 1

/* A CSR matrix: host struct of device pointers.  vals may be NULL where a
 * call reads only the pattern. */
typedef struct csrad_csr {
    int32_t nrows, ncols, nnz;
    int32_t dtype;
    const int32_t *rowptr;
    const int32_t *colind;
    const void *vals;
} csrad_csr;

/* Human-readable name of a status code (static storage). */
const char *csr_status_string(int status);

/* Traversal plan for the row-parallel dense-operand kernels (SpMM forward
 * and backward).  row_stride = 0 visits rows in natural order.  With
 * row_stride > 0, rows are visited as tiles of the (p, q) grid
 * row = p * row_stride + q: a tile is row_tile consecutive q for one p, and the tiles of one q-range are visited for every p
 * before the next q-range.  For operators whose long-range couplings sit at
 * a fixed row offset (structured grids) this keeps the dense rows that
 * neighbouring tiles share in cache.  The plan changes only the order of
 * work, never a result.  csr_pattern_stats gives the inputs an autotuner
 * needs to propose plans. */
typedef struct csrad_plan {
    int32_t row_stride;
    int32_t row_tile;
} csrad_plan;

/* Pattern statistics (synchronises): stats_host[0] = longest row,
 * [1] = bandwidth max |col - row|, [2] = number of non-empty rows,
 * [3] = nnz.  work needs 32 bytes. */
int csr_pattern_stats(const csrad_csr *A, int64_t *stats_host, void *work,
                      size_t work_bytes, void *stream);

/* ---------------------------------------------------------------------
 * SpMV (Section 3.1.1; Table 1, SpMV row).
 * csr_spmv_fwd: y[nrows] = A x[ncols].
 * csr_spmv_bwd: VJP with upstream gradient gy[nrows]:
 *   gx[ncols] = A^T gy, and gvals[nnz] with gvals[e] = gy[row e] x[col e].
 *   With At (pattern of A^T from csr_transpose, vals ignored) and perm,
 *   both gradients come from one deterministic gather over A^T; with At
 *   NULL the A^T product is formed by atomic accumulation (summation
 *   order then varies between runs).
 * ------------------------------------------------------------------- */
int csr_spmv_fwd(const csrad_csr *A, const void *x, void *y, void *stream);
int csr_spmv_bwd(const csrad_csr *A, const csrad_csr *At, const int32_t *perm,
                 const void *x, const void *gy, void *gx, void *gvals,
                 void *stream);
/* csr_spmv_bwd_split: the same VJP (Section 3.1.1) with both gradients
 * requested and At/perm given, formed as g_x by the gather over A^T and
 * g_vals row-wise over A (coalesced writes), the two passes sharing one
 * launch.  Results are bit-identical to csr_spmv_bwd with At.  Returns
 * CSRAD_EINVAL when At, perm (nnz > 0), gx or gvals is missing or At does
 * not match A's shape. */
int csr_spmv_bwd_split(const csrad_csr *A, const csrad_csr *At,
                       const int32_t *perm, const void *x, const void *gy,
                       void *gx, void *gvals, void *stream);

/* ---------------------------------------------------------------------
 * SpDMM, sparse times dense (Section 3.1.3; Table 1, SpDMM row).
 * csr_spmm_fwd: C[nrows x k] = A B[ncols x k].
 * csr_spmm_bwd: VJP with upstream gradient gC[nrows x k]:
 *   gB[ncols x k] = A^T gC (gather over the transpose At/perm, which the
 *   paper also uses: sparse transpose, then the forward product), and
 *   gvals[e] = <gC[row e, :], B[col e, :]> (the masked product (gC B^T)
 *   on A's pattern).  At/perm are required when gB is requested; with
 *   both outputs requested one fused pass over A^T produces both.
 *   plan (may be NULL: natural order) orders the rows of A (forward) or of
 *   A^T (backward); its row_stride must be 0 or in [1, rows] and row_tile
 *   positive when row_stride is.
 * ------------------------------------------------------------------- */
int csr_spmm_fwd(const csrad_csr *A, int32_t k, const void *B, int64_t ldb,
                 void *C, int64_t ldc, const csrad_plan *plan, void *stream);
int csr_spmm_bwd(const csrad_csr *A, const csrad_csr *At, const int32_t *perm,
                 int32_t k, const void *B, int64_t ldb, const void *gC,
                 int64_t ldgc, void *gB, int64_t ldgb, void *gvals,
                 const csrad_plan *plan, void *stream);

/* ---------------------------------------------------------------------
 * Sparse transpose (Section 3.1.3, used by every A^T product).
 * Pattern of A^T: rowptrT[ncols+1], colindT[nnz] (source rows ascending
 * within each column, so the result is canonical CSR), and perm[nnz] with
 * valsT[t] = vals[perm[t]].  Integer output is bit-exact and identical
 * between runs.
 * ------------------------------------------------------------------- */
int csr_transpose_workspace(const csrad_csr *A, size_t *bytes);
int csr_transpose(const csrad_csr *A, int32_t *rowptrT, int32_t *colindT,
                  int32_t *perm, void *work, size_t work_bytes, void *stream);
/* csr_transpose_noalloc: csr_transpose without a workspace argument, for
 * callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid hipMalloc).  The scratch space
 * lives in a static device array of csr_noalloc_scratch_bytes() bytes
 * (64 MiB), which every GPU the library runs on holds until the process
 * ends; the call allocates nothing.  Returns CSRAD_EWORKSPACE when the
 * transpose of A would need more (csr_transpose_workspace(A) above the
 * limit: roughly 2.5 nnz + 2 ncols int32 values over 64 MiB), CSRAD_EHIP if
 * the array's device address cannot be obtained.  Outputs as csr_transpose
 * (bit-identical).  Every call on one GPU shares the one array: calls that
 * overlap on one GPU (other streams, other host threads) race; calls
 * ordered on one stream are safe. */
int csr_transpose_noalloc(const csrad_csr *A, int32_t *rowptrT, int32_t *colindT,
                          int32_t *perm, void *stream);
size_t csr_noalloc_scratch_bytes(void);
/* Values of A^T in A^T's order: valsT[t] = vals[perm[t]] (nnz entries). */
int csr_transpose_vals(const csrad_csr *A, const int32_t *perm, void *valsT,
                       void *stream);

/* ---------------------------------------------------------------------
 * SpSpMM, sparse times sparse (Section 3.1.2; Table 1, SpSpMM row).
 * C = A B with A (m x n), B (n x p).  The pattern of C is structural:
 * (i,j) is stored when some k has (i,k) in A and (k,j) in B, even if the
 * sum cancels; column indices ascending.
 * csr_spgemm_symbolic: C_rowptr[m+1] and *C_nnz_host (synchronises).
 *   The rows are classified by their number of products; with bins_host
 *   non-NULL (CSRAD_SPGEMM_BINS int32 entries) the class boundaries are
 *   returned in the same synchronisation.
 * csr_spgemm_fwd: C_colind[nnz(C)] and C_vals[nnz(C)] given C_rowptr.
 *   Each C_ij sums A_ik B_kj in a fixed order (deterministic): k in A's
 *   row order for rows with more than 64 products; for shorter rows the
 *   products meeting at j are added by a fixed lane tree over A's row
 *   order (the row merge).
 *   bins_host may be NULL (the rows are classified again); non-NULL, it
 *   must be what csr_spgemm_symbolic returned for the same A and B, with
 *   `work` that symbolic call's workspace, unchanged since: the
 *   classification is then reused and empty classes launch nothing.
 * csr_spgemm_bwd: VJP with upstream gradient gC on pat(C) (Table 1):
 *   gA = (V B^T) on pat(A), gB = (A^T V) on pat(B).  C carries the
 *   pattern of C (vals ignored); At/permA (transpose of A) are required
 *   when gB is requested.
 * ------------------------------------------------------------------- */
#define CSRAD_SPGEMM_BINS 9
int csr_spgemm_workspace(const csrad_csr *A, const csrad_csr *B, size_t *bytes);
int csr_spgemm_symbolic(const csrad_csr *A, const csrad_csr *B,
                        int32_t *C_rowptr, int64_t *C_nnz_host,
                        int32_t *bins_host, void *work, size_t work_bytes,
                        void *stream);
int csr_spgemm_fwd(const csrad_csr *A, const csrad_csr *B,
                   const int32_t *C_rowptr, int32_t *C_colind, void *C_vals,
                   const int32_t *bins_host, void *work, size_t work_bytes,
                   void *stream);
int csr_spgemm_bwd(const csrad_csr *A, const csrad_csr *B,
                   const csrad_csr *At, const int32_t *permA,
                   const csrad_csr *C, const void *gC, void *gA, void *gB,
                   void *stream);

/* ---------------------------------------------------------------------
 * Sparse + sparse (Section 3.1.4; Table 1, Sp + Sp rows).
 * C = alpha A + beta B for A and B of the same shape (m x n).  The
 * pattern of C is the union of the two patterns, kept structurally: (i,j)
 * is stored when A or B stores it, even if the sum cancels; column
 * indices ascending.
 * csr_spadd_symbolic: C_rowptr[m+1] and *C_nnz_host (synchronises).
 *   Reads only the patterns.  `work` holds csr_spadd_workspace bytes.
 * csr_spadd_fwd: C_vals[nnz(C)] and, unless C_colind is NULL, C_colind,
 *   given C_rowptr from csr_spadd_symbolic for the same patterns (with
 *   the patterns unchanged, a later call may pass C_colind = NULL to
 *   recompute values only).  Each value is alpha A_ij + beta B_ij
 *   evaluated in float64 with the two products and the sum rounded
 *   separately (an absent term is left out), then rounded once to the
 *   value type.  With both inputs empty C is empty and C_vals may be
 *   NULL.
 * csr_spadd_bwd: VJP with upstream gradient gC on pat(C) (Table 1):
 *   gA = alpha V on pat(A), gB = beta V on pat(B), each product rounded
 *   once from float64.  A, B and C carry patterns (vals ignored) and one
 *   dtype.  Either gradient may be NULL.
 * alpha and beta are constants of the call (not differentiated).
 * ------------------------------------------------------------------- */
int csr_spadd_workspace(const csrad_csr *A, const csrad_csr *B, size_t *bytes);
int csr_spadd_symbolic(const csrad_csr *A, const csrad_csr *B,
                       int32_t *C_rowptr, int64_t *C_nnz_host, void *work,
                       size_t work_bytes, void *stream);
int csr_spadd_fwd(const csrad_csr *A, const csrad_csr *B, double alpha,
                  double beta, const int32_t *C_rowptr, int32_t *C_colind,
                  void *C_vals, void *stream);
int csr_spadd_bwd(const csrad_csr *A, const csrad_csr *B, const csrad_csr *C,
                  double alpha, double beta, const void *gC, void *gA,
                  void *gB, void *stream);

/* ---------------------------------------------------------------------
 * Sparse triangular solve (Section 3.1.5; Table 1, SpSolve row).
 * T is square, lower (lower = 1) or upper (lower = 0) triangular with a
 * stored, non-unit diagonal (a stored entry on the other side of the
 * diagonal is a precondition violation).
 * csr_trisolve_analyze: level sets of the solve's dependency graph.  A
 *   row that reads no other row is on level 0; otherwise it is one above
 *   the highest level among the rows it reads.  Writes level_of_row[n],
 *   level_ptr[nlevels+1], level_rows[n] (rows ascending within a level)
 *   and *nlevels_host (synchronises); level_ptr_host (host memory for
 *   n+1 entries, may be NULL) receives level_ptr's nlevels+1 entries in
 *   the same synchronisation.  Tt is the pattern of T^T (csr_transpose).
 *   Returns CSRAD_ESINGULAR if a diagonal is missing.
 * csr_trisolve_fwd: x = T^{-1} b, level by level.  level_ptr (device) and
 *   level_ptr_host (its host copy, nlevels+1 entries) come from
 *   csr_trisolve_analyze; the host copy schedules the launches (large
 *   levels as grid launches, runs of small levels in one workgroup).
 * csr_trisolve_bwd: VJP with upstream gradient gx: gb = T^{-T} gx (the
 *   solve with T^T runs over Tt/perm and the levels of T in reverse), and
 *   gvals[(i,j)] = -gb_i x_j on pat(T).  gb is required.
 * ------------------------------------------------------------------- */
int csr_trisolve_workspace(const csrad_csr *T, size_t *bytes);
int csr_trisolve_analyze(const csrad_csr *T, int32_t lower,
                         const csrad_csr *Tt, int32_t *level_of_row,
                         int32_t *level_ptr, int32_t *level_rows,
                         int32_t *nlevels_host, int32_t *level_ptr_host,
                         void *work, size_t work_bytes, void *stream);
int csr_trisolve_fwd(const csrad_csr *T, int32_t lower, int32_t nlevels,
                     const int32_t *level_ptr_host, const int32_t *level_ptr,
                     const int32_t *level_rows, const void *b, void *x,
                     void *stream);
int csr_trisolve_bwd(const csrad_csr *T, int32_t lower, const csrad_csr *Tt,
                     const int32_t *perm, int32_t nlevels,
                     const int32_t *level_ptr_host, const int32_t *level_ptr,
                     const int32_t *level_rows, const void *x, const void *gx,
                     void *gb, void *gvals, void *stream);

/* ---------------------------------------------------------------------
 * Conjugate gradients as device-resident steps (the Krylov iteration of
 * Section 4.3) and the reverse mode of each step.  A is square; vectors
 * have A's value type; dot products accumulate in float64 with a fixed
 * reduction order, so steps are bit-reproducible.  scal (8 float64 on the
 * device) carries the solver scalars, step (1 int32 on the device) the
 * step index, hist (hist_cap x 5 float64, may be NULL) receives per step
 * (rho_t, sigma_t, alpha_t, rho_{t+1}, beta_t).  No call synchronises.
 * csr_cg_init: x = 0, r = p = b, rho = b.b, step = 0.
 * csr_cg_step: q = A p; alpha = rho/(p.q); x += alpha p; r -= alpha q;
 *   beta = (r.r)/rho; p = r + beta p (alpha = beta = 0 once rho is 0).
 *   p_save (p before the step) and r_save (r after it) may be NULL.
 * csr_cg_step_bwd: undoes one step in reverse given that step's p_t, q_t,
 *   r_{t+1} and hist record, the upstream gradient gR of r_{t+1} (may be
 *   NULL) and the running adjoints xb, rb, pb, qb (vectors) and scal
 *   (reverse slots); accumulates the value gradient into gvals (q = A p
 *   contributes qb_i p_j at (i,j)).  At: the transpose of A with its
 *   values (csr_transpose / csr_transpose_vals, same dtype as A).
 * csr_cg_finish_bwd: gb = rb + pb + 2 rhob b after the first step is undone.
 * The workspace (csr_cg_workspace) holds block partial sums.
 * ------------------------------------------------------------------- */
int csr_cg_workspace(const csrad_csr *A, size_t *bytes);
int csr_cg_init(const csrad_csr *A, const void *b, void *x, void *r, void *p,
                double *scal, int32_t *step, void *work, size_t work_bytes,
                void *stream);
int csr_cg_step(const csrad_csr *A, void *x, void *r, void *p, void *q,
                void *p_save, void *r_save, double *scal, int32_t *step,
                double *hist, int32_t hist_cap, void *work, size_t work_bytes,
                void *stream);
int csr_cg_step_bwd(const csrad_csr *A, const csrad_csr *At, const void *p,
                    const void *q, const void *r1, const double *step_hist,
                    const void *gR, void *xb, void *rb, void *pb, void *qb,
                    double *scal, void *gvals, void *work, size_t work_bytes,
                    void *stream);
int csr_cg_finish_bwd(const csrad_csr *A, const void *b, const void *rb,
                      const void *pb, const double *scal, void *gb,
                      void *stream);

/* ---------------------------------------------------------------------
 * Preconditioned CG (Section 4.3) with float64 vectors and dot products
 * over float32 or float64 matrix values, device-resident like csr_cg_*.
 * kind: 0 Jacobi (dinv = 1/diag(A) from csr_diag_inv), 1 factor
 * (z = L^{-T} L^{-1} r with L lower triangular, its transpose Lt/perm and
 * its level sets from csr_trisolve_analyze; when Lt->vals is non-NULL it
 * holds L^T's values (csr_transpose_vals, same dtype as L) and perm is not
 * read), 2 none, 3 inverse factor (the form learned in Section 4.3:
 * M = L L^T approximates A^{-1} and z = L (L^T r) by two sparse products;
 * L any square sparse matrix, Lt/perm as for kind 1, no level sets:
 * nlevels 0 and NULL level pointers).  scal (16 float64 on
 * the device): [0] r.z, [1] p.q, [2] alpha, [3] beta, [4] ||b||,
 * [5] ||r||/||b||, [6] done flag, [7] breakdown flag, [8] steps taken,
 * [9] tolerance.  A step that finds ||r||/||b|| <= tol sets done; p.q not
 * positive and finite, or a non-finite r.z, sets breakdown and done.
 * Steps after done change nothing, so the host may run steps in chunks
 * and read scal in between.  hist (hist_cap float64, may be NULL)
 * receives ||r||/||b|| per step.
 * csr_pcg_workspace sizes the workspace shared by init and the steps; for
 * the factor kind pass L and its levels, for the inverse-factor kind L
 * with nlevels 0 and NULL (else NULL, 0, NULL).  init copies
 * A into an ELL layout inside the workspace and, when every level of L
 * has at least 1024 rows, L and L^T by level as well (for the inverse
 * factor, L and L^T whole; values included: call init again after A's or
 * L's values change); the steps read those copies.  A segment whose ELL copy would exceed twice the matrix's nnz is
 * read from the CSR arrays instead.
 * ------------------------------------------------------------------- */
int csr_pcg_workspace(const csrad_csr *A, const csrad_csr *L, int32_t nlevels,
                      const int32_t *level_ptr_host, size_t *bytes);
int csr_diag_inv(const csrad_csr *A, double *dinv, void *stream);
int csr_pcg_init(const csrad_csr *A, int32_t kind, const double *dinv,
                 const csrad_csr *L, const csrad_csr *Lt, const int32_t *perm,
                 int32_t nlevels, const int32_t *level_ptr_host,
                 const int32_t *level_ptr, const int32_t *level_rows,
                 const double *b, double *x, double *r, double *z, double *p,
                 double tol, double *scal, void *work, size_t work_bytes,
                 void *stream);
int csr_pcg_step(const csrad_csr *A, int32_t kind, const double *dinv,
                 const csrad_csr *L, const csrad_csr *Lt, const int32_t *perm,
                 int32_t nlevels, const int32_t *level_ptr_host,
                 const int32_t *level_ptr, const int32_t *level_rows,
                 double *x, double *r, double *z, double *p, double *q,
                 double *scal, double *hist, int32_t hist_cap, void *work,
                 size_t work_bytes, void *stream);

/* ---------------------------------------------------------------------
 * Learned preconditioner network (float32 tensors, hidden width 32).
 * csr_dense_fwd: Y (n x 32) = act([X1 X2] W + b) on bf16 matrix cores with
 *   float32 accumulation; X1 (n x K1, leading dim ld1), X2 (n x K2, may be
 *   absent with K2 = 0), W ((K1+K2) x 32 row-major, float32, rounded to
 *   bf16 for the products), b (32, may be NULL), relu = 1 or identity;
 *   K1 + K2 <= 64.
 * csr_dense_bwd: with G = dY * act'(Y): dX1, dX2 = G W^T (may be NULL),
 *   dW = [X1 X2]^T G, db = column sums of G (may be NULL; need the
 *   workspace of csr_dense_workspace; deterministic).
 * csr_mpnn_prep: for A (float32, square) and Lpat = tril(A)'s pattern:
 *   ahat = D^{-1/2} A D^{-1/2} on A's pattern, ahatL the same on Lpat,
 *   dsqrt = sqrt(diag A), X0 (n x 16) node inputs [1, sum |ahat_offdiag|,
 *   sum ahat_offdiag, (row length - 1)/8, then for the neighbours j < i
 *   and j > i in turn: sum ahat_ij, sum |ahat_ij|, count/8; 0...].
 * csr_mpnn_readout: L on Lpat from the per-entry network output t:
 *   L_ij = sqrt(A_ii) ahat_ij (1 + t_ij) for j < i and
 *   L_ii = sqrt(A_ii) (softplus(t_ii + c) + delta), so diag(L) > 0.
 * csr_mpnn_readout_bwd: gt = dL/dt given gL.
 * ------------------------------------------------------------------- */
int csr_dense_workspace(int32_t n, size_t *bytes);
int csr_dense_fwd(int32_t n, int32_t K1, const float *X1, int64_t ld1,
                  int32_t K2, const float *X2, int64_t ld2, const float *W,
                  const float *b, int32_t relu, float *Y, void *stream);
int csr_dense_bwd(int32_t n, int32_t K1, const float *X1, int64_t ld1,
                  int32_t K2, const float *X2, int64_t ld2, const float *W,
                  const float *Y, const float *dY, int32_t relu, float *dX1,
                  float *dX2, float *dW, float *db, void *work,
                  size_t work_bytes, void *stream);
int csr_mpnn_prep(const csrad_csr *A, const csrad_csr *Lpat, float *ahat,
                  float *ahatL, float *dsqrt, float *X0, void *stream);
int csr_mpnn_readout(const csrad_csr *Lpat, const float *ahatL,
                     const float *dsqrt, const float *t, float c, float delta,
                     float *Lv, void *stream);
int csr_mpnn_readout_bwd(const csrad_csr *Lpat, const float *ahatL,
                         const float *dsqrt, const float *t, float c,
                         const float *gL, float *gt, void *stream);

/* ---------------------------------------------------------------------
 * Batched operators over a block-diagonal CSR matrix (many independent
 * sparse matrices of uneven sizes concatenated along the diagonal; block b
 * owns rows and columns [block_rowptr[b], block_rowptr[b+1])).  The ops
 * are those of Sections 3.1.1 (SpMV), 3.1.3 (SpDMM) and 3.1.5 (SpSolve),
 * each as ONE persistent launch over a work queue of tasks.
 *
 * A plan (csr_batch_plan_build) cuts every block into row-aligned tasks of
 * about `budget` path items (rows + stored entries), orders the blocks by
 * that cost, largest first, and gives each task its block's traversal
 * variant:
 *   -1  leave the block out (its rows are not written),
 *    0  automatic (from the block's mean row length),
 *   1..7 row-split, 2^(v-1) lanes per row (SpMV; the SpMM kernels use
 *        one 16-lane group per row for any v != 8),
 *    8  merge-path: the task's merge path of row ends and entries is cut
 *        into equal pieces, one per thread (SpMV) or per 16-lane group
 *        (SpMM); rows cut by a piece boundary are completed from the
 *        pieces' partial sums in piece order (for blocks with very uneven
 *        rows; merge tasks take merge_budget(budget) =
 *        clamp(budget/4, 256, 4096) path items),
 *    9  rows staged 256 at a time in LDS (short rows; SpMV).
 * Every variant is deterministic; a variant's result does not depend on
 * the other blocks of the batch.  budget <= 0 makes one task per block
 * (the triangular solves need that).  A plan covers the rows of the matrix
 * it was built on: the forward ops take a plan of A, the backward ops a
 * plan of A^T (csr_transpose of a block-diagonal matrix is block-diagonal
 * with the same blocks).
 *
 * csr_batch_plan_workspace: bytes of device memory the plan keeps (task
 *   records, queue counters, block_rowptr); the caller owns it and keeps
 *   it alive while the plan is used.
 * csr_batch_plan_build: fills *plan (a host struct pointing into `work`);
 *   block_rowptr_host (nblocks+1 host int32, from 0 to A's rows,
 *   non-decreasing) and variant_host (nblocks host int32, may be NULL =
 *   automatic) are read during the call, which synchronises the stream.
 * The queue counters of a plan are shared by its launches: launches that
 * use one plan must be ordered on one stream.
 * ------------------------------------------------------------------- */
typedef struct csrad_batch_plan {
    int32_t nrows;   /* rows of the matrix the plan was built on */
    int32_t nblocks;
    int32_t ntasks;
    int32_t cus;     /* compute units; a launch keeps as many workgroups on each as
                        the kernel's occupancy allows */
    const void *tasks;           /* device, inside the plan workspace */
    void *counters;              /* device, inside the plan workspace */
    const int32_t *block_rowptr; /* device copy, inside the plan workspace */
} csrad_batch_plan;

int csr_batch_plan_workspace(const csrad_csr *A, int32_t nblocks, int32_t budget,
                             size_t *bytes);
int csr_batch_plan_build(const csrad_csr *A, int32_t nblocks,
                         const int32_t *block_rowptr_host,
                         const int32_t *variant_host, int32_t budget, void *work,
                         size_t work_bytes, csrad_batch_plan *plan, void *stream);

/* y = A x (plan of A).  Same arguments as csr_spmv_fwd. */
int csr_batch_spmv_fwd(const csrad_csr *A, const csrad_batch_plan *plan,
                       const void *x, void *y, void *stream);
/* VJP of y = A x over A^T (At/perm from csr_transpose; planT a plan of At):
 * gx = A^T gy, gvals[e] = gy[row e] x[col e]; either output may be NULL. */
int csr_batch_spmv_bwd(const csrad_csr *A, const csrad_csr *At,
                       const int32_t *perm, const csrad_batch_plan *planT,
                       const void *x, const void *gy, void *gx, void *gvals,
                       void *stream);
/* C = A B (plan of A); k a multiple of 4 (float32) or 2 (float64), B and
 * C 16-byte aligned with 16-byte aligned rows. */
int csr_batch_spmm_fwd(const csrad_csr *A, const csrad_batch_plan *plan,
                       int32_t k, const void *B, int64_t ldb, void *C,
                       int64_t ldc, void *stream);
/* VJP of C = A B in one pass over A^T (planT a plan of At): gB = A^T gC,
 * gvals[e] = <gC[row e,:], B[col e,:]>; either output may be NULL. */
int csr_batch_spmm_bwd(const csrad_csr *A, const csrad_csr *At,
                       const int32_t *perm, const csrad_batch_plan *planT,
                       int32_t k, const void *B, int64_t ldb, const void *gC,
                       int64_t ldgc, void *gB, int64_t ldgb, void *gvals,
                       void *stream);
/* Value gradients alone, row-wise over A with a plan of A (the other half
 * of a backward split into an A^T product over At's plan, computed with
 * gx / gB only, and this coalesced pass; the results equal the fused
 * pass's): csr_batch_sddmv: gvals[e] = gy[row e] x[col e];
 * csr_batch_sddmm: gvals[e] = <gC[row e,:], B[col e,:]> (k and alignment
 * as csr_batch_spmm_fwd). */
int csr_batch_sddmv(const csrad_csr *A, const csrad_batch_plan *plan,
                    const void *x, const void *gy, void *gvals, void *stream);
int csr_batch_sddmm(const csrad_csr *A, const csrad_batch_plan *plan, int32_t k,
                    const void *B, int64_t ldb, const void *gC, int64_t ldgc,
                    void *gvals, void *stream);
/* Triangular solves per block (plan built with budget <= 0).  The level
 * sets of the whole block-diagonal T come from csr_trisolve_analyze;
 * csr_batch_levels writes, into a caller workspace of
 * csr_batch_levels_workspace bytes, where each block's rows sit in each
 * level (asynchronous).  csr_batch_trisolve_fwd: x = T^{-1} b, one
 * workgroup per block running its levels in order.
 * csr_batch_trisolve_bwd: gb = T^{-T} gx over Tt/perm with the levels in
 * reverse, then gvals[(i,j)] = -gb_i x_j on pat(T) (gvals may be NULL). */
int csr_batch_levels_workspace(int32_t nblocks, int32_t nlevels, size_t *bytes);
int csr_batch_levels(const csrad_batch_plan *plan, int32_t nlevels,
                     const int32_t *level_ptr, const int32_t *level_rows,
                     void *work, size_t work_bytes, void *stream);
int csr_batch_trisolve_fwd(const csrad_csr *T, const csrad_batch_plan *plan,
                           int32_t nlevels, const int32_t *level_rows,
                           const void *levels_work, size_t levels_bytes,
                           const void *b, void *x, void *stream);
int csr_batch_trisolve_bwd(const csrad_csr *T, const csrad_csr *Tt,
                           const int32_t *perm, const csrad_batch_plan *plan,
                           int32_t nlevels, const int32_t *level_rows,
                           const void *levels_work, size_t levels_bytes,
                           const void *x, const void *gx, void *gb,
                           void *gvals, void *stream);
/* Level-synchronous batched solves: ONE cooperative launch over the whole
 * block-diagonal T (every workgroup resident at once; the levels of the
 * batch, from csr_trisolve_analyze on T, are the unions of the blocks'
 * levels).  Each level's rows are shared by all workgroups, one row per
 * thread, with a grid barrier between levels, so large blocks use the whole
 * chip instead of one workgroup each.  csr_batch_trisolve_levels_fwd:
 * x = T^{-1} b.  csr_batch_trisolve_levels_bwd: gb = T^{-T} gx over Tt/perm
 * with the levels in reverse, then gvals[(i,j)] = -gb_i x_j on pat(T)
 * (gvals may be NULL).  level_ptr (nlevels+1) and level_rows are device
 * arrays.  Returns CSRAD_EHIP if the runtime refuses the cooperative launch
 * (the chip cannot hold the grid). */
int csr_batch_trisolve_levels_fwd(const csrad_csr *T, int32_t nlevels,
                                  const int32_t *level_ptr, const int32_t *level_rows,
                                  const void *b, void *x, void *stream);
int csr_batch_trisolve_levels_bwd(const csrad_csr *T, const csrad_csr *Tt,
                                  const int32_t *perm, int32_t nlevels,
                                  const int32_t *level_ptr, const int32_t *level_rows,
                                  const void *x, const void *gx, void *gb, void *gvals,
                                  void *stream);
/* Incomplete Cholesky IC(0) per block (the factor the batched solves
 * take; Saad, Section 10.3): Alow is tril(A) with its values (diagonal
 * stored and last in every row); Lvals (nnz(Alow)) receives L on the same
 * pattern with L_ij = (A_ij - sum_{k<j} L_ik L_jk) / L_jj and
 * L_ii = sqrt(A_ii - sum_{k<i} L_ik^2), sums over the columns stored in
 * both rows, entries of a row in column order.  Rows run level by level
 * (the levels of the lower solve on Alow's pattern, as for
 * csr_batch_trisolve_fwd; plan built with budget <= 0).  A non-positive
 * pivot leaves NaN in that diagonal and in every entry computed from it. */
int csr_batch_ic0(const csrad_csr *Alow, const csrad_batch_plan *plan,
                  int32_t nlevels, const int32_t *level_rows,
                  const void *levels_work, size_t levels_bytes, void *Lvals,
                  void *stream);

/* ---------------------------------------------------------------------
 * The vector and scalar steps of a short PCG unroll and their reverse
 * mode, for training a preconditioner on the residual-history loss of
 * Section 4.3, l = sum_i w_i ||r_i|| / ||b|| (the products q = A p and
 * the preconditioner z = M^{-1} r are the library's other calls).  Vectors
 * of n entries of `dtype`; scalars float64 on the device; dot products
 * summed in a fixed order (bit-reproducible).  `work` holds
 * csr_pcgl_workspace(n) bytes; none of the calls synchronises.
 * csr_pcgl_start:  scal[0] = rho_0 = b.z_0, scal[1] = ||b||.
 * csr_pcgl_res_fwd: sigma = p.q, alpha = rho/sigma, r1 = r - alpha q,
 *   nr = ||r1||, acc1 = acc + w nr / bnorm; scal[0..2] = sigma, alpha, nr.
 * csr_pcgl_res_bwd: given the adjoints gr1 (may be NULL) and gacc1 of r1
 *   and acc1, writes those of r, q, p and rho (acc's adjoint is gacc1).
 * csr_pcgl_dir_fwd: rho1 = r1.z1, beta = rho1/rho, p1 = z1 + beta p.
 * csr_pcgl_dir_bwd: given gp1 (may be NULL) and grho1 (may be NULL),
 *   writes the adjoints of r1, z1, p and rho.
 * csr_pcgl_start_bwd: gz0 = grho0 b + gp0 (either may be NULL).
 * ------------------------------------------------------------------- */
int csr_pcgl_workspace(int32_t n, size_t *bytes);
int csr_pcgl_start(int32_t n, int32_t dtype, const void *b, const void *z,
                   double *scal, void *work, size_t work_bytes, void *stream);
int csr_pcgl_res_fwd(int32_t n, int32_t dtype, const void *p, const void *q,
                     const void *r, const double *rho, double w,
                     const double *bnorm, const double *acc, void *r1,
                     double *scal, double *acc1, void *work, size_t work_bytes,
                     void *stream);
int csr_pcgl_res_bwd(int32_t n, int32_t dtype, const void *p, const void *q,
                     const void *r1, const double *rho, const double *scal,
                     double w, const double *bnorm, const void *gr1,
                     const double *gacc1, void *gr, void *gq, void *gp,
                     double *grho, void *work, size_t work_bytes, void *stream);
int csr_pcgl_dir_fwd(int32_t n, int32_t dtype, const void *r1, const void *z1,
                     const double *rho, const void *p, double *rho1, void *p1,
                     void *work, size_t work_bytes, void *stream);
int csr_pcgl_dir_bwd(int32_t n, int32_t dtype, const void *r1, const void *z1,
                     const double *rho, const void *p, const double *rho1,
                     const void *gp1, const double *grho1, void *gr1, void *gz1,
                     void *gp, double *grho, void *work, size_t work_bytes,
                     void *stream);
int csr_pcgl_start_bwd(int32_t n, int32_t dtype, const void *b, const void *gp0,
                       const double *grho0, void *gz0, void *stream);

/* ---------------------------------------------------------------------
 * Pattern check: rowptr monotone from 0 to nnz, colind in [0, ncols),
 * strictly ascending within each row.  *first_bad_row_host receives the
 * first offending row or -1 (synchronises).  Returns CSRAD_EPATTERN if a
 * row is malformed.  work needs 8 bytes.
 * ------------------------------------------------------------------- */
int csr_validate(const csrad_csr *A, int32_t *first_bad_row_host, void *work,
                 size_t work_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CSRAD_H */
