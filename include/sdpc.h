/*
 * sdpc.h -- C ABI of the matrix-completion primal-dual interior-point hot
 * path on one AMD MI355X (gfx950).
 *
 * Problem (Section 1 of Yamashita & Nakata, "Fast implementation for
 * semidefinite programs with positive matrix completion"):
 *
 *   (P)  min A_0 . X   s.t.  A_k . X = b_k (k = 1..m),  X psd
 *   (D)  max sum_k b_k z_k   s.t.  sum_k A_k z_k + Y = A_0,  Y psd
 *
 * The primal matrix is kept only on the extended sparsity pattern E (the
 * chordal extension of the aggregate pattern, Section 2.1); its
 * max-determinant completion X^ is applied through the Cholesky factor of
 * its inverse, X^{-1} = Lhat Lhat^T, built clique by clique (Algorithm 1),
 * and Y through its sparse Cholesky factor Y = N N^T.  Both factors share
 * one storage layout (Section 3.1).  The Schur complement matrix
 * B_pq = A_p . (X^ A_q Y^{-1}) (eq. SCM, evaluated as in eq. newSCM2) is
 * assembled on the device and factorised densely in FP64.
 *
 * Conventions for every call:
 *   - All functions return an sdpc_status (0 = SDPC_OK, negative = error);
 *     nothing throws across the ABI and the library never aborts.  On error
 *     a detail string is kept on the handle (sdpc_last_error).
 *   - "Device" pointers are HIP device allocations owned by the caller
 *     (e.g. torch tensors); "host" pointers are ordinary host memory.
 *   - All device work is enqueued on the hipStream_t given at create.
 *     Calls marked (async) return before the work is done; the others
 *     synchronise that stream before returning.
 *   - The library allocates all of its device workspace in sdpc_create and
 *     frees it in sdpc_destroy; no call allocates in between.
 *   - A handle is not thread-safe: use one handle per host thread.
 *   - "E-vectors" hold a symmetric matrix on E in the library's storage
 *     order (sdpc_get_pattern reports, for every stored position, its row
 *     and column in ORIGINAL indices, or -1 for padding).  Padding slots
 *     are ignored on input and written as zero on output.
 */
#ifndef SDPC_H
#define SDPC_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sdpc_handle sdpc_handle;

typedef enum {
    SDPC_OK = 0,
    SDPC_E_ARG = -1,        /* invalid argument (null pointer, bad size, bad index)      */
    SDPC_E_PATTERN = -2,    /* structure not supported (e.g. a clique larger than 64)    */
    SDPC_E_NOT_PD = -3,     /* a matrix that must be positive definite is not            */
    SDPC_E_HIP = -4,        /* a HIP runtime call failed                                 */
    SDPC_E_MAXITER = -5,    /* iteration limit reached before the stopping test held     */
    SDPC_E_STAGNATION = -6, /* step lengths collapsed; no further progress               */
    SDPC_E_NUMERIC = -7,    /* NaN or Inf met                                            */
    SDPC_E_OOM = -8         /* device allocation failed at create                        */
} sdpc_status;

/* The problem in standard form.  Host memory, read only during sdpc_create.
 * Matrix A_k (k = 0..m) is the list of lower-triangle triplets
 * (row[t], col[t], val[t]) for t in [ptr[k], ptr[k+1]); indices are 0-based
 * with row >= col; duplicates are summed; the upper triangle is implied by
 * symmetry. */
typedef struct {
    int32_t n;                 /* order of X and Y                        */
    int32_t m;                 /* number of constraints                   */
    const int64_t *ptr;        /* m + 2 offsets                           */
    const int32_t *row;
    const int32_t *col;
    const double *val;
    const double *b;           /* length m                                */
} sdpc_problem;

/* Parameters.  The paper leaves beta, gamma, the initial point and the
 * stopping rule open (Section 2.2); the defaults are the readings the CPU
 * oracle uses as well. */
typedef struct {
    double gap_tol;            /* relative gap  |P-D| / max(1,(|P|+|D|)/2)         (1e-7)  */
    double feas_tol;           /* primal / dual infeasibility tolerance            (1e-7)  */
    double beta_feas;          /* centring parameter once feasible                 (0.1)   */
    double beta_infeas;        /* centring parameter before                        (0.2)   */
    double gamma;              /* fraction of the maximal step                     (0.9)   */
    double lambda0;            /* X0 = Y0 = lambda0 I, z0 = 0                      (100)   */
    int32_t max_iter;          /*                                                  (100)   */
    int32_t ordering;          /* 0 natural, 1 minimum degree, 2 user_perm         (0)     */
    int32_t block_width;       /* widest storage block (columns), 1..32            (32)    */
    int32_t verbose;           /* 1: one line per iteration on stderr              (0)     */
    int32_t pool_lds_bytes;    /* LDS budget per wave of the Y factorisation's pending-update
                                  pool; larger pools live in device memory; 0 keeps them
                                  there always                                    (32768)  */
    int32_t solve_kernel;      /* substitution walk forming X^ and Y^{-1}: 0 picks the
                                  matrix-core walk when the blocks fit it, 1 always the
                                  generic walk                                    (0)      */
    int32_t factorization;     /* how X^ is applied: 0 through X^{-1} = Lhat Lhat^T built by
                                  Algorithm 1 (Section 3.1); 1 through the earlier sparse
                                  factorisation X^ = L^T D L (eq. sparse_fact, Section 2.1),
                                  substituting with the sparse L^{-1} around the block
                                  diagonal D                                       (0)      */
    int32_t merge_siblings;    /* storage blocks: 1 also merges consecutive sibling
                                  subtrees of the elimination tree whose rows below the
                                  block do not grow (explicit zeros only: E and every
                                  result are unchanged, the block walks get shorter);
                                  0 merges chains only                             (1)      */
    int32_t dual_points;       /* dual step length (Step 3): test points per round of the
                                  parallel positive-definiteness search; 0 takes 511 points
                                  then 384 (two rounds, made for one instance alone on the
                                  GPU); otherwise rounds of this many points (2..511) until
                                  the bracket is narrower than 5e-5 relative       (0)      */
    int32_t chol_kernel;       /* SCM Cholesky (type (i) of Section 3.1): 0 one launch, a
                                  dataflow over the 64-column blocks (tiles updated
                                  left-looking, each block's tiles finished together);
                                  1 one launch per 64-column block; both give the same
                                  factor up to rounding order                      (0)      */
    const int32_t *user_perm;  /* ordering == 2: user_perm[i] = original index eliminated
                                  i-th (host, read at create)                              */
} sdpc_params;

/* Result of sdpc_solve / sdpc_step. */
typedef struct {
    int32_t status;            /* sdpc_status of the solve                                 */
    int32_t iters;             /* iterations performed                                     */
    double pobj, dobj;         /* A_0 . X and b . z                                        */
    double rel_gap, pinf, dinf;
    double mu, alpha_p, alpha_d, beta;   /* last iteration                                 */
    double t_scm_ms;           /* device time: Y factor, Algorithm 1, solves, SCM (sum)    */
    double t_chol_ms;          /* device time: SCM Cholesky and SCE solve (sum)            */
    double t_pmatrix_ms;       /* device time: dX on E and the step lengths (sum)          */
    double t_total_ms;         /* wall time of the call                                    */
    double t_potrf_ms;         /* device time of the SCM Cholesky alone (sum)              */
    int32_t n_potrf;           /* SCM Cholesky factorisations timed in t_potrf_ms          */
    int32_t pad_;
    size_t device_bytes;       /* device workspace held by the handle                      */
} sdpc_result;

/* Defaults listed above. */
sdpc_params sdpc_default_params(void);

/* Sizes found by the symbolic phase. */
typedef struct {
    int64_t nslot;             /* stored positions of the shared factor layout            */
    int64_t nnzE;              /* lower-triangle entries of E (diagonal included)          */
    int32_t ncliques;          /* l, the number of cliques (supernodes)                    */
    int32_t nblocks;           /* storage blocks                                           */
    int32_t max_clique;        /* max |C_r|                                                */
    int32_t max_block_rows, max_block_cols;
    int32_t nfwd, nbwd;        /* live rows of the forward / backward substitutions         */
    int32_t hadamard;          /* 1 when every A_k (k >= 1) is one diagonal entry          */
    int64_t sum_clique;        /* sum_r |C_r|                                              */
    /* Limits the structure must respect (sdpc_create fails with SDPC_E_PATTERN
     * beyond them) and the device memory sdpc_create will ask for. */
    int32_t limit_clique;      /* largest clique the clique kernels take (64)              */
    int32_t limit_panel;       /* largest storage panel h x w in doubles (4096)            */
    int32_t limit_m;           /* most constraints (65535)                                 */
    int32_t pad_;
    int64_t device_bytes;      /* workspace of sdpc_create: three dense n x n matrices
                                  (X^, Y^{-1}, a product), the (m+1) x m SCM, 1024
                                  candidate factors of nslot doubles, and small arrays    */
} sdpc_analysis;

/* Host-only symbolic phase (Section 2.1, Section 3.1); touches no device
 * and may run on a machine without a GPU.  info (host) receives the sizes.
 * Optional host outputs (NULL to skip): perm (n): elimination order,
 * perm[i] = original index eliminated i-th; cptr (ncliques + 1), cidx
 * (sum_clique), nS (ncliques): the cliques C_r in original indices, S_r
 * being the first nS[r] members.  Call once with NULL arrays to size them. */
sdpc_status sdpc_analyze(const sdpc_problem *prob, const sdpc_params *params, sdpc_analysis *info,
                         int32_t *perm, int64_t *cptr, int32_t *cidx, int32_t *nS);

/* Symbolic phase (Section 2.1, Section 3.1): aggregate pattern, ordering,
 * chordal extension, elimination tree, supernodes as the clique sequence
 * C_1..C_l with S_r / U_r, storage blocks, all index maps; then allocates
 * the device workspace and uploads the problem.  params may be NULL
 * (defaults).  On success *out owns everything; on failure *out is NULL. */
sdpc_status sdpc_create(const sdpc_problem *prob, const sdpc_params *params,
                        hipStream_t stream, sdpc_handle **out);

/* Full solve from the initial point of Section 2.2, Step 0, to the stopping
 * test (Steps 1-4 repeated).  res (host) receives the outcome.  The final
 * iterate stays on the handle (sdpc_get_solution). */
sdpc_status sdpc_solve(sdpc_handle *h, sdpc_result *res);

/* Reset the iterate to Step 0's initial point. (async) */
sdpc_status sdpc_reset(sdpc_handle *h);

/* One iteration (Steps 1-4) from the handle's current iterate.  Returns
 * SDPC_OK after an update; res->status is SDPC_OK when the stopping test
 * already held (no update made).  Unless the gap is already near the stopping
 * tolerance, the next iteration's Schur complement phase is left enqueued on
 * the handle's stream when it returns (later calls on the handle are ordered
 * after it). */
sdpc_status sdpc_step(sdpc_handle *h, sdpc_result *res);

/* The Schur complement matrix at a given state: Y = N N^T (sparse
 * Cholesky), Lhat by Algorithm 1 from Xbar, the columns of X^ and Y^{-1}
 * by sparse substitutions, then B_pq = A_p . (X^ A_q Y^{-1}) (eq. SCM /
 * eq. newSCM2).  d_Xbar_E, d_Y_E: E-vectors (device, length nslot).  d_B:
 * device m x m column-major, leading dimension ldb >= m; the lower triangle
 * (row >= col, constraint order) is written, the strict upper triangle is
 * left untouched.  factor != 0 additionally overwrites that lower triangle
 * with the Cholesky factor R of B (B = R R^T).  Errors found on the device
 * (a non-positive-definite clique block of Xbar, a Y that is not positive
 * definite, a B that is not) are reported by the return value, so the call
 * synchronises the stream before returning. */
sdpc_status sdpc_scm(sdpc_handle *h, const double *d_Xbar_E, const double *d_Y_E,
                     double *d_B, int64_t ldb, int32_t factor);

/* Dense FP64 Cholesky B = R R^T in place (lower triangle of a column-major
 * m x m device matrix, ldb >= m, 0 <= m <= the handle's number of
 * constraints, whose workspace it uses; SDPC_E_ARG otherwise), the
 * factorisation used for the SCM (type (i) of Section 3.1).  The strict upper
 * triangle is not referenced.
 * Returns SDPC_E_NOT_PD (with the pivot in the detail string) if B is not
 * positive definite.  Synchronises. */
sdpc_status sdpc_potrf(sdpc_handle *h, double *d_B, int64_t ldb, int32_t m);

/* Pattern of the storage layout: the extended sparsity pattern E (the chordal
 * extension of the aggregate pattern, Section 2.1) in the storage order of
 * the factors, which Lhat and N share (Section 3.1).  *nslot receives the number of stored
 * positions.  iE / jE (host, length nslot, may be NULL) receive, for each
 * stored position, its (row, col) in ORIGINAL indices with row >= col in the
 * elimination order's sense (the position's own row/column), or -1/-1 for a
 * padding slot outside E.  perm (host, length n, may be NULL) receives the
 * elimination order: perm[i] = original index eliminated i-th.  ncliques
 * (may be NULL) receives the number of cliques (supernodes) l. */
sdpc_status sdpc_get_pattern(const sdpc_handle *h, int64_t *nslot, int32_t *iE, int32_t *jE,
                             int32_t *perm, int32_t *ncliques);

/* Clique sequence C_1..C_l (original indices): cptr (host, l + 1) and cidx
 * (host, sum |C_r|), with S_r the first nS[r] members of C_r.  Any array may
 * be NULL. */
sdpc_status sdpc_get_cliques(const sdpc_handle *h, int64_t *cptr, int32_t *cidx, int32_t *nS);

/* Current iterate (Xbar on E, Y, z) of the method of Section 2.2 in the
 * notation of problems (P) and (D): Xbar_E, Y_E (E-vectors) and z (length m);
 * device pointers, any may be NULL.  After a failed sdpc_step or sdpc_solve
 * this is the last iterate that was accepted: a step whose factorisations
 * reported an error, or whose step lengths collapsed, changes none of X, Y and
 * z.  Synchronises. */
sdpc_status sdpc_get_solution(const sdpc_handle *h, double *d_Xbar_E, double *d_Y_E, double *d_z);

/* Replace the current iterate (device pointers; none may be NULL). (async) */
sdpc_status sdpc_set_state(sdpc_handle *h, const double *d_Xbar_E, const double *d_Y_E,
                           const double *d_z);

/* Factors in the storage layout (E-vectors in the elimination order):
 * d_N (Y = N N^T, Section 3.1 type (v)), d_Lhat (X^{-1} = Lhat Lhat^T,
 * Algorithm 1).  After sdpc_scm both belong to the state it was given.
 * Inside sdpc_step / sdpc_solve the next X's Lhat is formed while the dual
 * step runs, and the next iteration's Schur complement phase is usually
 * enqueued before the step returns, so after an iteration d_Lhat belongs to
 * the new X and d_N to the new Y or to the Y the iteration started from; call
 * sdpc_scm with the state from sdpc_get_solution for factors of one iterate.  With
 * factorization = 1, d_Lhat receives L^{-1} of eq. sparse_fact instead.
 * Either may be NULL.  Synchronises. */
sdpc_status sdpc_get_factors(const sdpc_handle *h, double *d_N, double *d_Lhat);

/* Dense X^ (max-determinant completion, Section 2.1) and Y^{-1} formed by the
 * last SCM evaluation: sdpc_scm, or after sdpc_step / sdpc_solve the Schur
 * complement phase of the iterate the last iteration started from or, when the
 * next iteration's phase was enqueued ahead (the usual case), of the new iterate.  n x n
 * column-major in the ELIMINATION order (position i is original index
 * perm[i]).  Either may be NULL.  Synchronises. */
sdpc_status sdpc_get_dense(const sdpc_handle *h, double *d_Xhat, double *d_Yinv);

/* Max-determinant positive definite completion X^ of the handle's CURRENT
 * Xbar (Section 2.1; X^ agrees with Xbar on E and its inverse vanishes off
 * E): Algorithm 1 gives X^{-1} = Lhat Lhat^T (or, with factorization = 1, the
 * factorisation of eq. sparse_fact), then X^ e_k by sparse substitutions for
 * every k (type (iv) of Section 3.1).  d_Xhat (device, n x n column-major in
 * ORIGINAL indices, may be NULL to only form it) receives X^.  Returns
 * SDPC_E_NOT_PD if a clique block Xbar(C_r, C_r) is not positive definite.
 * Overwrites the buffers sdpc_get_dense and sdpc_get_factors read.
 * Synchronises. */
sdpc_status sdpc_complete_dense(sdpc_handle *h, double *d_Xhat);

/* Search direction of the last sdpc_step (Section 2.2, Step 2 with
 * eq. newdX2 and the clique-wise step of eq. primal_length2): d_dz (length
 * m), d_dX_E, d_dY_E (E-vectors), and the host scalars alpha (2 doubles:
 * alpha_p, alpha_d before the gamma factor).  Any may be NULL.  Synchronises. */
sdpc_status sdpc_get_direction(const sdpc_handle *h, double *d_dz, double *d_dX_E,
                               double *d_dY_E, double *alpha);

/* Device time (ms) of the kernels of the last sdpc_scm, split as
 * [Y factor, Algorithm 1, solves, SCM assembly, SCM Cholesky].  Host array
 * of 5.  Synchronises. */
sdpc_status sdpc_get_scm_timing(const sdpc_handle *h, double *ms5);

/* Batched solves: many independent SDPs of uneven sizes on one GPU, each solved
 * as by sdpc_solve (Section 2.2, Steps 0-4 with the Schur complement phase of
 * Section 3.1) while many are in flight at once.  The independent Schur
 * complement columns of the paper's parallel scheme (Section 3.2) become
 * independent instances here: host workers, one HIP stream each, take the
 * instances longest estimated work first; every handle is created before any
 * solve starts and released after all have finished; an instance retires as
 * soon as its own stopping test holds.  With autotune the storage-block width
 * (the tile width of the clique panels) is chosen per size class (largest
 * clique <= 8 / <= 16 / more, times n <= 200 / <= 500 / more) by timing real
 * iterations of the class's largest instance at widths 8, 16 and 32. */
typedef struct {
    int32_t workers;           /* host workers, one HIP stream each, 1..64           (8)  */
    int32_t autotune;          /* 1: choose the block width per size class            (1)  */
    int32_t tuned_width[9];    /* out: width chosen per class (3 x clique class + order
                                  class), 0 where no instance fell in the class          */
    int32_t dual_points;       /* dual_points of every instance whose params leave it 0:
                                  many instances share the GPU, so each searches the dual
                                  step with fewer points per round                    (32) */
    double tune_ms, create_ms, solve_ms, total_ms;   /* out: wall time of the phases        */
} sdpc_batch_options;

/* Defaults listed above. */
sdpc_batch_options sdpc_default_batch_options(void);

/* probs (host, count), params (host, count, may be NULL for defaults; each
 * instance's own user_perm is honoured), opt (host, may be NULL; receives the
 * tuning outcome and times), results (host, count): each instance's outcome as
 * from sdpc_solve (results[i].status its status).  d_z (host array of count
 * device pointers, may be NULL, entries may be NULL): z of each instance
 * (length m_i).  The device is the current one.  Returns SDPC_OK when every
 * instance solved, else the status of the first one that did not (the others
 * are still solved); the detail is in sdpc_last_error(NULL).  Synchronises. */
sdpc_status sdpc_batch_solve(int32_t count, const sdpc_problem *probs, const sdpc_params *params,
                             sdpc_batch_options *opt, sdpc_result *results, double *const *d_z);

/* Centring: Newton steps of Step 2 of Section 2.2 from the handle's current
 * iterate with the centring target beta mu replaced by the fixed mu (> 0), so
 * that the iterate converges to the point of the central path with
 * X^ Y = mu I, A(X) = b and sum_k z_k A_k + Y = A_0 (step lengths as in Steps
 * 3-4).  The stopping test of Step 1 is not applied.  Stops after max_steps
 * steps or once a step moves z by at most tol relative to max(1, max|z|).
 * steps (host, optional) receives the steps taken, last_rel_step (host,
 * optional) that relative move.  A failed step leaves the iterate as it was
 * and returns its status.  Synchronises. */
sdpc_status sdpc_center(sdpc_handle *h, double mu, int32_t max_steps, double tol, int32_t *steps,
                        double *last_rel_step);

/* Derivatives of a loss L(X, z) at the handle's current iterate, taken to be a
 * point of the central path (sdpc_center): the central point is a smooth
 * function of (b, A_0) for fixed mu, and differentiating its three equations
 * leads to the Schur complement matrix B of eq. SCM (not part of the paper's
 * method; the same matrix and substitutions are reused).  Inputs: d_GL_E
 * (device E-vector), the symmetric gradient of L with respect to X, which must
 * vanish off the aggregate sparsity pattern (entries there are ignored: the
 * completion X^ equals Xbar only on E); d_dLdz (device, length m, may be NULL
 * for 0), the gradient with respect to z.  Outputs (device):
 *   d_gb   (length m)  dL/db = lambda = B^{-1} (h + dL/dz), h_p = A_p . (X^ G_L Y^{-1})
 *   d_gC_E (E-vector)  dL/dA_0 = sym(X^ (sum_k lambda_k A_k - G_L) Y^{-1}) on E, in the
 *                      Frobenius product: a change of A_0 by a symmetric dA_0
 *                      supported on E changes L by sum_ij (dL/dA_0)_ij (dA_0)_ij.
 * Overwrites the buffers sdpc_get_dense and sdpc_get_factors read.  Returns
 * SDPC_E_NOT_PD if a factorisation fails.  Synchronises. */
sdpc_status sdpc_adjoint(sdpc_handle *h, const double *d_GL_E, const double *d_dLdz, double *d_gb,
                         double *d_gC_E);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the dense
 * FP64 Cholesky of sdpc_potrf, B = R R^T in place on the lower triangle of a
 * column-major m x m device matrix (ldb >= max(1, m)), without a handle.  It
 * calls no hipMalloc, hipFree or allocating library routine: its workspace
 * (64 KiB of parked diagonal factors and a failure flag) is one fixed device
 * array per GPU, held from the first call on that GPU until the process ends.
 * Limit: m <= 65535 (SDPC_E_ARG beyond it, with the reason in
 * sdpc_last_error(NULL)).  All work is enqueued on `stream` (its device is the
 * one used; NULL: the current device's default stream).
 * d_info (device, optional): with d_info != NULL the call is asynchronous and
 * *d_info receives 0, or 1 + the failing pivot if B is not positive definite
 * (-1 if an internal hand-over wait ran out); with d_info == NULL the call
 * synchronises the stream and returns SDPC_E_NOT_PD on a failed pivot.
 * Every call on one GPU shares that GPU's workspace: calls that overlap on one
 * GPU (other streams, other host threads) race and must be serialised by the
 * caller. */
sdpc_status sdpc_potrf_static(double *d_B, int64_t ldb, int32_t m, int32_t *d_info, hipStream_t stream);

const char *sdpc_status_string(sdpc_status s);
/* Detail of the last error of handle h; with h == NULL, of the last failed
 * call made without a handle on this host thread. */
const char *sdpc_last_error(const sdpc_handle *h);
void sdpc_destroy(sdpc_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* SDPC_H */
