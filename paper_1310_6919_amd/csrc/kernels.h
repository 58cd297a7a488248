// Device data structures and kernel launchers (host-callable).
//
// Lhat, N and every E-vector share one storage layout (Section 3.1):
// block b owns columns [bl_first[b], bl_first[b+1]) and rows
// bl_rows[bl_rptr[b] .. bl_rptr[b+1]) (own columns first); its panel is the
// h x w column-major array at offset bl_off[b].
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace sdpc {

// Detail string of the last failed call made without a handle, per host thread
// (what sdpc_last_error(NULL) returns).
std::string &unbound_error();
void set_unbound_error(const std::string &msg);

// Copy count doubles from global memory to LDS, issuing U loads per thread before
// any LDS store so that the loads overlap instead of waiting one by one.
template <int U = 8>
__device__ inline void stage_lds(double *dst, const double *__restrict__ src, int count) {
    for (int base = threadIdx.x; base < count; base += U * blockDim.x) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * blockDim.x;
            v[u] = i < count ? src[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * blockDim.x;
            if (i < count) dst[i] = v[u];
        }
    }
}

struct DevStruct {
    int n = 0, m = 0, nb = 0, ncl = 0;
    int64_t nslot = 0;
    int max_h = 0, max_w = 0, max_clique = 0;
    int64_t max_panel = 0;              // max over blocks of h * w
    // blocks
    const int *bl_first = nullptr;      // nb + 1
    const int64_t *bl_rptr = nullptr;   // nb + 1
    const int *bl_rows = nullptr;       // sum h
    const int64_t *bl_off = nullptr;    // nb + 1
    const int *bl_subfirst = nullptr;   // nb
    const int *bl_fslot = nullptr;      // sum h: forward solve slot of each row (-1: none)
    const int *bl_bslot = nullptr;      // sum h: backward solve slot of each row (-1: none)
    // the single-product walks (blocks <= 32 wide, <= 64 high): per block 64 entries
    // for its rows r in the order (r % 4) * 16 + r / 4, -1 beyond the block: forward
    // slot, first block that updates the row, backward slot
    const int *wk_fs = nullptr, *wk_fb = nullptr, *wk_bs = nullptr;
    const int64_t *bl_dinv = nullptr;   // nb + 1: offsets of the w x w diagonal-block inverses
    const int64_t *up_ptr = nullptr;    // nb + 1: update pairs of each block
    const int *up_pair = nullptr;       // (a | c << 16), a >= c, indices into the non-own rows
    const int *up_slot = nullptr;       // target slot, -1 if not stored (value is exactly zero)
    // pending updates of the one-wave factorisation live in slots: an update's code is
    // (slot << 1) | (first update of the slot in block order), or -1.  With u_pool the
    // nU slots are a pool in LDS reused after their panel is consumed; otherwise one
    // slot per target entry, in global memory, nU per candidate.  Slot nU - 2 stays
    // zero, slot nU - 1 takes the results that update nothing.
    int64_t nU = 0;
    int u_pool = 0;
    const int *su_rows = nullptr;       // nb x 8 x 64 x 4: the slot each panel entry adds (row i, column k
                                        // at [k / 4][i][k % 4]; nU - 2 where none and outside)
    // the one-wave factorisation's per-block sizes (w, h, offset, 0) and, for each of the
    // wc_rt (wc_rt + 1) / 2 lower tile pairs of L21 L21^T, lane l and element r, the
    // update code of the entry (16 ti + 4 r + l / 16, 16 tj + l % 16), or that of slot
    // nU - 1 (int4 per lane)
    const int *wc_meta = nullptr;
    const int *wc_up = nullptr;
    int wc_rt = 2;
    int nfwd = 0, nbwd = 0;             // live rows of the multi-right-hand-side substitutions
    int wk_nfwd = 0, wk_nbwd = 0;       // and of the single-product walks
    const int *col_block = nullptr;     // n: block of every column
    const int *slot_row = nullptr;      // nslot: row position of an E slot, -1 on padding
    const int *slot_col = nullptr;      // nslot: column position of an E slot, -1 on padding
    // cliques (fundamental supernodes)
    const int *cl_first = nullptr;      // ncl + 1
    const int64_t *cl_ptr = nullptr;    // ncl + 1: offsets into cl_rows
    const int *cl_rows = nullptr;       // C_r in positions, ascending
    const int64_t *cl_map_ptr = nullptr;// ncl + 1
    const int *cl_map = nullptr;        // packed lower-triangle slots of C_r x C_r, column by column
    // E-vector weights: 1 (diagonal), 2 (off-diagonal), 0 (padding); also the E mask
    const double *wE = nullptr;
    // assembly: slot s collects sum_t asm_val[t] * coef(asm_k[t]) for t in asm_ptr[s]..
    const int64_t *asm_ptr = nullptr;   // nslot + 1
    const int *asm_k = nullptr;
    const double *asm_val = nullptr;
    // constraints k = 0..m: lower entries (pi >= pj positions), slot, value * multiplicity
    const int64_t *con_ptr = nullptr;   // m + 2
    const int *con_pi = nullptr, *con_pj = nullptr, *con_slot = nullptr;
    const double *con_val = nullptr;
    // constraints longer than kConLong entries (when any is): the entries of each
    // constraint cut into chunks of kConChunk, chunk c belonging to ch_con[c] and
    // starting at entry ch_beg[c]; constraint k's chunks are ch_ptr[k] .. ch_ptr[k+1]-1
    int con_chunks = 0;                 // 0: one wave per constraint instead
    const int *ch_con = nullptr, *ch_ptr = nullptr;
    const int64_t *ch_beg = nullptr;
    const double *b = nullptr;          // m
    // Schur complement: single diagonal entry per A_k (max-cut form)
    int hadamard = 0;
    const int *had_pos = nullptr;       // m
    const double *had_val = nullptr;    // m
    // general path: A_q restricted to its nonzero columns K_q, full symmetric CSC
    const int64_t *kq_ptr = nullptr;    // m + 1: columns of A_q are kq_col[kq_ptr[q]..]
    const int *kq_col = nullptr;
    const int64_t *aq_cptr = nullptr;   // (sum |K_q|) + 1, indexed by the global column id
    const int *aq_row = nullptr;
    const double *aq_val = nullptr;
    // union support S of A_1..A_m (full symmetric), grouped by row
    int64_t nS = 0;
    const int64_t *S_rowptr = nullptr;  // n + 1
    const int *S_col = nullptr;         // column of each support entry
    const int64_t *am_ptr = nullptr;    // m + 1: entries of A_p as (support index, value)
    const int64_t *am_sidx = nullptr;
    const double *am_val = nullptr;
    // aggregate pattern, full symmetric CSC by columns with E slots (for G and dY)
    const int64_t *ag_cptr = nullptr;   // n + 1
    const int *ag_row = nullptr;
    const int *ag_slot = nullptr;
    // the same pattern by groups of 32 consecutive columns: the union of the rows of a
    // group (padded to a multiple of 4) and, per union row and column of the group, the
    // slot of the entry (-1: none); every group is a dense product on the MFMA over its
    // union, kZmRows union rows at a time.
    // A group whose union exceeds kZmSplit rows is cut into pieces of kZmPiece union
    // rows, each a group of its own (split K): zg_col gives a group's columns (32 zg_col
    // ..), zg_piece its piece (-1: a whole group).  The products of the pieces go to
    // zpart (npiece x 32 x n) and are added in piece order into Z; the right-hand-side
    // form simply has one partial sum per group.
    int nzg = 0;                        // groups, pieces counted one by one
    const int64_t *zg_ptr = nullptr;    // nzg + 1: offsets into zg_rows (zg_slot: 32 per row)
    const int *zg_rows = nullptr;
    const int *zg_slot = nullptr;
    const int *zg_col = nullptr;        // nzg
    const int *zg_piece = nullptr;      // nzg
    int nzg_mma = 0;
    const int *zg_mma = nullptr;        // groups on the MFMA path
    int npiece = 0, nzsplit = 0;        // pieces; column groups that were cut
    const int *zs_g = nullptr;          // nzsplit: the column group
    const int *zs_ptr = nullptr;        // nzsplit + 1: its pieces
    double *zpart = nullptr;            // npiece x 32 x n work
    // general path, column-compressed form (k_scm_cc.hip): A_q = U_q + U_q^T + D_q with
    // U_q the strict triangle (upper or lower, whichever has the smaller column union C
    // over all q) and D_q the diagonal
    int cc = 0;                         // 1: the column-compressed form is used
    int nc = 0;                         // |C|
    const int *ccol = nullptr;          // nc positions
    const double *ucat = nullptr;       // n x (m nc) column-major: U_1(:, C) .. U_m(:, C)
    int nds = 0;                        // positions holding a diagonal entry of some A_q
    const int *ds = nullptr;            // nds
    const double *dmat = nullptr;       // nds x m column-major: D_q(ds[i])
    // the constraints with a diagonal part when there are at most kDqFew of them (ndq
    // of them, listed in dq), else ndq = -1
    int ndq = -1;
    const int *dq = nullptr;
    int64_t nseg = 0;                   // rows of A_1 .. A_m (full symmetric), in order
    const int *seg_q = nullptr;         // nseg
    const int *seg_row = nullptr;       // nseg
    const int64_t *seg_ptr = nullptr;   // nseg + 1: entries (seg_col, seg_val) of each row
    const int *seg_col = nullptr;
    const double *seg_val = nullptr;
    const int *pos = nullptr;           // n: position (elimination order) of every original index
    int solve_generic = 0;              // 1: the substitutions always take the generic walk
};
constexpr int kZmRows = 128;
constexpr int kDqFew = 8;
constexpr int kZmSplit = 512, kZmPiece = 128;

// ---- assembly and vectors (k_vec.hip)
// out[s] = sum_t asm_val[t] * coef_k  + c1 * in1[s]; coef_0 = a0, coef_k = -y[k-1]
void launch_assemble(const DevStruct &d, const double *y, double a0, double c1, const double *in1,
                     double *out, hipStream_t st);
size_t metrics_work_doubles(const DevStruct &d);   // work of launch_metrics and launch_rhs
constexpr int kConLong = 256, kConChunk = 1024;
// With chunks (d.con_chunks > 0): out[k] = b_k - coef sum_e con_val[e] v(e) + (add ? add[k] : 0)
// over the entries of constraint k, v(e) = v[con_slot[e]] (an E-vector) or, dense,
// v(pi, pj) of an n x n matrix; the chunk sums in work + 8 kMetricsGroups + m.
// Returns false (nothing launched) without chunks.
bool launch_con_chunks(const DevStruct &d, bool dense, const double *v, double coef, const double *add,
                       double *out, double *work, hipStream_t st);
// scal[...] <- pobj, dobj, max|r|, max|G|, X.Y, also G_E (see k_vec.hip)
void launch_metrics(const DevStruct &d, const double *X, const double *Y, const double *z,
                    double *G, double *scal, double *work, hipStream_t st);
// out = x + scale * alpha[0] * dx when flags[0..nflag) are all zero and alpha[0] (and
// alpha2[0] when given) are positive, else out = x; out may be x
void launch_axpy_checked(int64_t len, const double *x, const double *dx, const double *alpha, const double *alpha2,
                         double scale, const int *flags, int nflag, double *out, hipStream_t st);
// out = pool + sel[0] * len (ncand vectors of length len; sel[0] a device double,
// the index; negative or >= ncand: out untouched)
void launch_copy_selected(int64_t len, const double *pool, const double *sel, int ncand, double *out,
                          hipStream_t st);
// out = a + b elementwise (b == nullptr: out = a)
void launch_add(int64_t len, const double *a, const double *b, double *out, hipStream_t st);
// out(i, j) = in(pos[i], pos[j]) for dense n x n column-major matrices
void launch_unpermute(const DevStruct &d, const double *in, double *out, hipStream_t st);
void launch_init_point(const DevStruct &d, double lambda, double *X, double *Y, double *z,
                       hipStream_t st);
void launch_mask_E(const DevStruct &d, double *v, hipStream_t st);

// ---- factorisations (k_factor.hip)
// Y = N N^T (supernodal); fail[0] = 0 or 1 + the failing block.  U: scratch of
// d.nU doubles per candidate (pending updates, when they are not kept in LDS); the
// dual step needs d.nU times the candidates of its largest round.
void launch_sn_chol(const DevStruct &d, const double *Y, double *L, double *U, double *work, int *fail,
                    hipStream_t st);
// work (doubles) of launch_sn_chol and launch_dual_step; LDS of their one-wave
// factorisation with a pool of npool update slots
size_t wave_chol_work_doubles(const DevStruct &d);
// rows of the one-wave factorisation's LDS panel, and its LDS bytes with a pool of npool slots
int wave_chol_rows(int max_h, int max_w);
size_t wave_chol_lds_bytes(int max_h, int max_w, int64_t npool);
// largest alpha in (0, 1] with Y + alpha dY positive definite: 'rounds' rounds of
// parallel factorisations of ntest[r] test points (log grid, then even grids inside
// the bracket), with gamma twins in the last round; the result is bracket[0] (a lower bound;
// bracket[1] an upper bound), bracket[3] the candidate holding the factor of
// Y + gamma bracket[0] dY (or -1), all on the device.  Only the gamma twins store
// their factors (in cand, d.nslot doubles each); the other tests keep nothing.
void launch_dual_step(const DevStruct &d, const double *Y, const double *dY, int rounds, const int *ntest,
                      double gamma, double *cand, double *U, double *work, int *fail, double *bracket,
                      hipStream_t st);
// candidates launched in a round (test points and their gamma twins)
int dual_step_candidates(int round, int rounds, const int *ntest);
// Dinv_b = L_bb^{-1} per storage block (w x w at bl_dinv); with G != nullptr also
// G_b = [L_bb^{-1}; P21_b L_bb^{-1}] (h x w), the one matrix of a block step of the
// single-product substitution walks, at G + 4096 b in the walks' lane order
// (walk_g_layout); needs w <= 32 and h <= 64.  With Dm (w x w blocks at bl_dinv)
// the forward operand's top block is Dm_b L_bb^{-1} instead, so the walks give
// L^{-T} Dm L^{-1} (the backward operand keeps L_bb^{-1})
void launch_dinv(const DevStruct &d, const double *L, double *Dinv, int *fail, hipStream_t st,
                 double *G = nullptr, const double *Dm = nullptr);
// Algorithm 1: Lhat from Xbar clique by clique; fail = 1 + clique on a non-PD block
void launch_algorithm1(const DevStruct &d, const double *Xbar, double *Lhat, int *fail,
                       hipStream_t st);
// the earlier factorisation X^ = L^T D L (eqs. sparse_fact, orig_L, orig_D): per
// clique the (C_r, S_r) columns of the unit-lower L^{-1} (factor layout) and D_r
// (w x w blocks at bl_dinv; the blocks must be zeroed once, entries between
// supernodes stay zero); needs every supernode inside one storage block; fail =
// 1 + clique on a non-PD block
void launch_ldl_cliques(const DevStruct &d, const double *Xbar, double *Linv, double *Dblk, int *fail,
                        hipStream_t st);
// eq. primal_length2: per-clique maximal step, then the minimum into *out
void launch_alpha_cliques(const DevStruct &d, const double *Xbar, const double *dX,
                          double *alpha_cl, double *alpha_hi, double *out, hipStream_t st);

// ---- sparse substitutions (k_solve.hip): out = (L L^T)^{-1}, n x n, full symmetric
int solve_tile_width(const DevStruct &d);
// out_f = L_f^{-T} L_f^{-1} (dense n x n) for one or two factors (L1 == nullptr: one);
// with Dm_f != nullptr (w x w blocks at bl_dinv, block diagonal over the supernodes)
// out_f = L_f^{-T} Dm_f L_f^{-1} instead: with L_f^{-1} of eq. sparse_fact as the
// factor this is X^ = L^T D L
// With G0 (and G1 for a second factor) from launch_dinv (given the same Dm) and every
// block at most 32 wide and 64 high, the walks take one product per block step
// (walk_g_ok); Dm then rides in G.
void launch_inverse_by_solves(const DevStruct &d, const double *L0, const double *Dinv0, double *out0,
                              const double *L1, const double *Dinv1, double *out1, hipStream_t st,
                              const double *Dm0 = nullptr, const double *Dm1 = nullptr,
                              const double *G0 = nullptr, const double *G1 = nullptr);
bool walk_g_ok(const DevStruct &d);

// ---- Schur complement (k_scm.hip)
void launch_scm_hadamard(const DevStruct &d, const double *Xh, const double *Yi, double *B,
                         int64_t ldb, hipStream_t st);
// general SCM, one column q at a time (kq_ptr_host: host mirror of kq_ptr); lower triangle
void launch_scm_general(const DevStruct &d, const int64_t *kq_ptr_host, const double *Xh,
                        const double *Yi, double *W, double *T, double *B, int64_t ldb,
                        hipStream_t st);
// col[p] = A_p . (X^ M Y^{-1}) for M on the aggregate pattern given as an E-vector
void launch_scm_extra_column(const DevStruct &d, const double *Mvec, const double *Xh,
                             const double *Yi, double *W, double *T, double *col, hipStream_t st);
// g_p = b_p - beta mu A_p . Y^{-1} + h_p
void launch_rhs(const DevStruct &d, const double *Yi, const double *h, double beta_mu, double *g,
                double *work, hipStream_t st);
// dX on E:  beta mu Y^{-1} - Xbar - sym(X^ dY Y^{-1}) with W = X^ dY (row-major)
void launch_dX(const DevStruct &d, const double *W, const double *Yi, const double *Xbar,
               double beta_mu, double *dX, hipStream_t st);
// Z = X^ M column-major (n x n) for M on the aggregate pattern (E-vector)
void launch_zcol(const DevStruct &d, const double *Xh, const double *Mvec, double *Z, hipStream_t st);
// max-cut form of the extra column: hcol[k] = (X^ M Y^{-1})(a_k, a_k); part: rhs_had_parts x n
int rhs_had_parts(const DevStruct &d);
void launch_rhs_hadamard(const DevStruct &d, const double *Mvec, const double *Xh, const double *Yi,
                         double *part, double *hcol, hipStream_t st);
// column-compressed general SCM (d.cc): B lower (ldb) from X^ and Y^{-1}; H: n x n
// workspace; work: cc_work_doubles(d), which keeps the blocks the extra column reuses
size_t cc_work_doubles(const DevStruct &d);
void launch_scm_cc(const DevStruct &d, const double *Xh, const double *Yi, double *H, double *work, double *B,
                   int64_t ldb, hipStream_t st);
// col[p] = A_p . (X^ M Y^{-1}) for M on the aggregate pattern, after launch_scm_cc on
// the same X^ and Y^{-1}; Z: n x n workspace
void launch_scm_cc_extra_column(const DevStruct &d, const double *Mvec, const double *Xh, const double *Yi,
                                double *Z, double *work, double *col, hipStream_t st);
// dX on E from Z = X^ dY (column-major): part holds 2 * dX_chunks * nslot doubles
int dX_chunks(const DevStruct &d);
void launch_dX_blocked(const DevStruct &d, const double *Z, const double *Yi, const double *Xbar,
                       double beta_mu, double *part, double *dX, hipStream_t st);
// W = X^ M (row-major n x n) for M on the aggregate pattern (E-vector)
void launch_dense_times_agg(const DevStruct &d, const double *Xh, const double *Mvec, double *W,
                            hipStream_t st);

// ---- dense FP64 Cholesky and SCE solve (k_dense.hip)
// Dense Cholesky of B (lower, column-major, leading dimension ldb); rows m..rows-1
// ride along (a right-hand side stored as row m ends as R^{-1} g).  fail gets
// pivot + 1 if B is not positive definite.  work: potrf_work_doubles(m) doubles.
//
// The backward solve's flags hold potrf_flag_count(m) ints, zero-initialised
// once; epoch must differ from every earlier call's on the same flags; fail gets
// -1 if an internal wait ran out.
int potrf_flag_count(int m);
size_t potrf_work_doubles(int m);
void launch_potrf(int m, double *B, int64_t ldb, double *work, int *fail, hipStream_t st);
void launch_potrf_rows(int m, int rows, double *B, int64_t ldb, double *work, int *fail, hipStream_t st);
// The same factorisation in one launch (dataflow over the 64-column blocks, every
// tile's left-looking updates kept in registers): flags hold
// potrf_flow_flag_count(m, rows) ints, zeroed once; epoch must differ from every
// earlier call's on the same flags; work: potrf_flow_work_doubles(m) doubles
int potrf_flow_flag_count(int m, int rows);
size_t potrf_flow_work_doubles(int m);
void launch_potrf_flow(int m, int rows, double *B, int64_t ldb, int *flags, double *work, int epoch, int *fail,
                       hipStream_t st);
// R^T x = u with R the factor left in B and u read with stride ustride
void launch_potrs_bwd(int m, const double *R, int64_t ldb, const double *u, int64_t ustride, double *x, int *flags,
                      int epoch, int *fail, hipStream_t st);
void launch_set_row(int m, const double *g, double *row, int64_t stride, hipStream_t st);

}  // namespace sdpc
