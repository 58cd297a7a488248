// Small dense Cholesky factorisations kept in registers.
//
// One row per lane, one wave (lane_bcast, elim_step_bcast, elim_lds): the
// one-wave sparse factorisations (Y = N N^T and the dual step's candidates, the
// clique-wise step-length test) and the diagonal blocks of the dense SCM Cholesky.
//
// chol_tile: a register-tiled Cholesky by one 256-thread workgroup, shared by
// Algorithm 1, the clique-wise step-length test for cliques of more than 32
// members and the tall supernodal panels of Y = N N^T.
//
// Thread t owns a TR x TC tile of the (NR x NC) working matrix, NR = (256 / JG) TR,
// NC = JG TC: rows i0 = TR (t / JG) + [0, TR), columns j0 = TC (t % JG) + [0, TC).
// Right-looking elimination, one pivot per step and one barrier per step:
//   * column k of the partially updated matrix (unscaled, zero above row k) and,
//     for the inverse, row k of the partially eliminated identity, sit in a
//     double-buffered LDS slot, written at the end of step k - 1 by the threads
//     that own them;
//   * every thread reads the pivot d = A(k, k), forms 1/sqrt(d) itself, scales
//     the few column / row values it needs and applies the rank-one update to its
//     whole tile.  Rows above k read zeros; the pivot column and the pivot row
//     are given a zero multiplier and scaled in place instead, so when the loop
//     ends the tiles hold L (lower triangle) and L^{-1} exactly, and nothing has
//     to leave the registers during the elimination.
// The pivot loop is unrolled by TC so every register index is a constant.
// Entries beyond the active order must be padded with the identity (square use)
// or zeros (panel rows), so that padded pivots are 1 and change nothing.
#pragma once
#include <hip/hip_runtime.h>

namespace sdpc {

// 1/sqrt(d) from the hardware estimate refined by two Newton steps
// (y <- y (3 - d y^2) / 2); sqrt(d) is then d / sqrt(d).  A short dependent
// chain compared with a correctly rounded square root followed by a division.
__device__ inline double rsqrt_newton(double d) {
    double y = __builtin_amdgcn_rsq(d);
    y = y * fma(-0.5 * d, y * y, 1.5);
    y = y * fma(-0.5 * d, y * y, 1.5);
    return y;
}

// The value of x held by lane `lane` of the wave (a uniform lane index), through
// two readlanes into scalar registers.
__device__ inline double lane_bcast(double x, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

// One step of a right-looking elimination held one row per lane: a[j] -= l *
// l(lane c0 + j) for k < j < 32.  The multipliers of the other rows arrive by
// readlane, eight at a time ahead of their fmas, so the readlanes do not wait on
// one another's scalar registers.
__device__ inline void elim_step_bcast(double (&a)[32], double l, int k, int c0) {
#pragma unroll
    for (int j0 = k + 1; j0 < 32; j0 += 8) {
        double lj[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) lj[u] = (j0 + u < 32) ? lane_bcast(l, c0 + j0 + u) : 0.0;
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (j0 + u < 32) a[j0 + u] = fma(-l, lj[u], a[j0 + u]);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Right-looking elimination of W columns held one row per lane, a[k] = A(lane,
// c0 + k), pivot k in lane c0 + k; lanes above the pivot get zero multipliers and
// row c0 + k gets sqrt(d).  A pivot that is not positive and finite leaves a NaN
// (or 0 * inf) on the diagonal.  The arithmetic and its order are those of one
// elim_step_bcast per column, but the bulk multipliers are broadcast through LDS:
// each step every lane stores its multiplier to Wl (64 doubles, 16-byte aligned,
// private to the wave) and reads back the ones it needs from uniform addresses.  A
// wave's LDS operations complete in order, so no wait separates the store from the
// reads.  Column k + 1 is updated first (its multiplier by readlane) and the next
// pivot's 1/sqrt is formed while the reads are in flight.  Fewer issue slots than
// readlanes for every multiplier (a wave alone on its SIMD is issue-bound there),
// at the cost of registers for the values in flight.
template <int W>
__device__ inline void elim_lds(double (&a)[W], int c0, double *Wl) {
    const int lane = threadIdx.x % 64;
    double inv = rsqrt_newton(lane_bcast(a[0], c0));
#pragma unroll
    for (int k = 0; k < W; ++k) {
        __builtin_amdgcn_sched_barrier(0);
        const double l = (lane >= c0 + k) ? a[k] * inv : 0.0;
        a[k] = l;
        if (k + 1 < W) {
            Wl[(lane - c0) & 63] = l;   // every lane: no branch
            a[k + 1] = fma(-l, lane_bcast(l, c0 + k + 1), a[k + 1]);
            double lj[W];
#pragma unroll
            for (int j = k + 2; j < W; ++j) lj[j] = Wl[j];
            __builtin_amdgcn_sched_barrier(0);
            inv = rsqrt_newton(lane_bcast(a[k + 1], c0 + k + 1));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = k + 2; j < W; ++j) a[j] = fma(-l, lj[j], a[j]);
        }
    }
    __builtin_amdgcn_sched_barrier(0);
}

template <int NR, int NC>
struct TileLds {
    double col[2][NR];   // column k of the working matrix (unscaled), rows 0..NR-1
    double row[2][NC];   // row k of the partially eliminated identity
};

// Loads TC consecutive doubles from LDS with 16-byte reads (TC even, aligned).
template <int N>
__device__ inline void lds_vec(const double *p, double (&v)[N]) {
    static_assert(N % 2 == 0, "even vector length");
#pragma unroll
    for (int u = 0; u < N; u += 2) {
        const double2 t = *reinterpret_cast<const double2 *>(p + u);
        v[u] = t.x;
        v[u + 1] = t.y;
    }
}

// Factorises the leading ncol columns.  a[][] holds the tile of the symmetric
// input (lower triangle; entries above it end up meaningless); with INV, r[][]
// must hold the tile of the identity.  On success a[][] holds the tile of L in
// its lower triangle (columns < ncol) and, with INV, r[][] the tile of L^{-1}.
// Returns false, uniformly, if a pivot is not positive and finite; *bad_pivot is
// its index.
template <int TR, int TC, int JG, bool INV>
__device__ inline bool chol_tile(double (&a)[TR][TC], double (&r)[TR][TC], int ncol,
                                 TileLds<(256 / JG) * TR, JG * TC> &sh, int *bad_pivot) {
    static_assert(!INV || TR == TC, "the inverse needs square tiles");
    static_assert(TC % TR == 0, "pivot rows must stay aligned with the unrolled columns");
    const int tid = threadIdx.x;
    const int ig = tid / JG, jg = tid % JG;
    const int i0 = TR * ig, j0 = TC * jg;
    __syncthreads();   // a previous call on the same buffers may still be reading them
    // publish column 0 and row 0 of the identity
    if (jg == 0) {
#pragma unroll
        for (int u = 0; u < TR; ++u) sh.col[0][i0 + u] = a[u][0];
    }
    if (INV && ig == 0) {
#pragma unroll
        for (int v = 0; v < TC; ++v) sh.row[0][j0 + v] = r[0][v];
    }
    __syncthreads();
    const int nkb = (ncol + TC - 1) / TC;
    for (int kb = 0; kb < nkb; ++kb) {
#pragma unroll
        for (int c = 0; c < TC; ++c) {
            const int k = TC * kb + c;
            if (k < ncol) {   // uniform
                const double *cb = sh.col[k & 1];
                const double d = cb[k];
                if (!(d > 0.0) || !isfinite(d)) {
                    *bad_pivot = k;
                    return false;   // uniform: every thread read the same pivot
                }
                const double inv = rsqrt_newton(d);
                double li[TR], lj[TC], rk[TC];
                lds_vec(cb + i0, li);
                lds_vec(cb + j0, lj);
                if (INV) lds_vec(sh.row[k & 1] + j0, rk);
                // the pivot row (row group k / TR, row c % TR) and the pivot column
                // (column group kb, column c) take no update; they are scaled below
                const int cr = c % TR;   // constants once the loop over c is unrolled
                const bool prow = (ig == k / TR), pcol = (jg == kb);
#pragma unroll
                for (int u = 0; u < TR; ++u) li[u] = (u == cr && prow) ? 0.0 : li[u] * inv;
#pragma unroll
                for (int v = 0; v < TC; ++v) lj[v] = (v == c && pcol) ? 0.0 : lj[v] * inv;
                if (INV) {
#pragma unroll
                    for (int v = 0; v < TC; ++v) rk[v] *= inv;
                }
#pragma unroll
                for (int u = 0; u < TR; ++u)
#pragma unroll
                    for (int v = 0; v < TC; ++v) a[u][v] = fma(-li[u], lj[v], a[u][v]);
                if (INV) {
#pragma unroll
                    for (int u = 0; u < TR; ++u)
#pragma unroll
                        for (int v = 0; v < TC; ++v) r[u][v] = fma(-li[u], rk[v], r[u][v]);
                }
                if (pcol) {   // column k of L (rows at and below k; zeros above)
#pragma unroll
                    for (int u = 0; u < TR; ++u) a[u][c] *= inv;
                }
                if (INV && prow) {   // row k of L^{-1}
#pragma unroll
                    for (int v = 0; v < TC; ++v) r[cr][v] *= inv;
                }
                // publish column k + 1 (rows above it zero) and row k + 1 of the inverse
                const int k1 = k + 1;
                const int cn = (c + 1) % TC;
                if (k1 < ncol) {
                    if (jg == k1 / TC) {
#pragma unroll
                        for (int u = 0; u < TR; ++u) sh.col[k1 & 1][i0 + u] = (i0 + u >= k1) ? a[u][cn] : 0.0;
                    }
                    if (INV && ig == k1 / TR) {
#pragma unroll
                        for (int v = 0; v < TC; ++v) sh.row[k1 & 1][j0 + v] = r[cn % TR][v];
                    }
                }
                __syncthreads();
            }
        }
    }
    return true;
}

}  // namespace sdpc
