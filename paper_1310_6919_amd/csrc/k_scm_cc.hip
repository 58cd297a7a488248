// Schur complement matrix for general constraint matrices (eq. SCM, with the
// dense columns of X^ and Y^{-1} as in eq. newSCM2), column-compressed form.
//
// Split every constraint matrix as A_q = U_q + U_q^T + D_q: U_q its strict
// triangle on the side whose column union C over all constraints is smaller,
// D_q its diagonal.  With T_q = X^ A_q Y^{-1},
//   <U_p, T_q>   = <X^ U_p, A_q Y^{-1}>          (columns C only)
//   <U_p, T_q^T> = <Y^{-1} U_p, A_q X^>         (columns C only)
//   <D_p, T_q>   = sum_a D_p(a) T_q(a, a),
//   T_q(a, a)    = [X^ U_q Y^{-1}](a, a) + [Y^{-1} U_q X^](a, a) + sum_i D_q(i) X^(a, i) Y^{-1}(a, i),
// so that, with the n x |C| blocks P_p = X^ U_p(:, C), P'_p = Y^{-1} U_p(:, C),
// Q_q = (A_q Y^{-1})(:, C) and Q'_q = (A_q X^)(:, C),
//   B_pq = <P_p, Q_q> + <P'_p, Q'_q> + sum_a D_p(a) T_q(a, a).
// P and P' for all constraints are two dense products X^ U_cat and Y^{-1} U_cat
// (U_cat = [U_1(:, C) ... U_m(:, C)], n x m|C|) on the FP64 MFMA; Q and Q' are
// sparse rows of A_q times the |C| x n rows Y^{-1}(C, :) and X^(C, :); the
// diagonal part is a Hadamard product restricted to the diagonal support times
// the matrix of the D_q.  The same blocks with A_q replaced by the dual
// residual G give A_p . (X^ G Y^{-1}) for the SCE right-hand side.
#include "kernels.h"

namespace sdpc {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// Rows C of two dense symmetric n x n matrices as |C| x n column-major blocks:
// YC(c, j) = Yi(ccol[c], j), XC(c, j) = Xh(ccol[c], j).
__global__ void __launch_bounds__(256)
k_gather_rows(int n, int nc, const int *__restrict__ ccol, const double *__restrict__ Yi,
              const double *__restrict__ Xh, double *__restrict__ YC, double *__restrict__ XC) {
    const int64_t total = int64_t(nc) * n;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
        const int c = int(i % nc);
        const int64_t j = i / nc;
        const int64_t src = ccol[c] + int64_t(n) * j;   // (ccol[c], j) = (j, ccol[c]) by symmetry
        YC[i] = Yi[src];
        XC[i] = Xh[src];
    }
}

// C_z = A_z B for z = blockIdx.z in {0, 1} (both column-major; A_z M x K, B K x N,
// C_z M x N).  64 x 64 output tile per workgroup, each of the four waves a 32 x 32
// quadrant of 2 x 2 MFMA tiles (16 x 16 x 4 FP64; lane l supplies A(l % 16, l / 16)
// and B(l / 16, l % 16), element r of the result is C(4 r + l / 16, l % 16)).  The
// operands of the next 16-wide step of K are loaded while the current one runs.
__global__ void __launch_bounds__(256)
k_gemm_nn(int M, int N, int K, const double *__restrict__ A0, const double *__restrict__ A1, int64_t lda,
          const double *__restrict__ Bm, int64_t ldb, double *__restrict__ C0, double *__restrict__ C1,
          int64_t ldc) {
    const double *A = blockIdx.z ? A1 : A0;
    double *C = blockIdx.z ? C1 : C0;
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    const int i0 = 64 * blockIdx.x + 32 * (wv & 1), j0 = 64 * blockIdx.y + 32 * (wv >> 1);
    int ra[2], cb[2];
    bool pa[2], pb[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int r = i0 + 16 * u + li, c = j0 + 16 * u + li;
        pa[u] = r < M;
        pb[u] = c < N;
        ra[u] = min(r, M - 1);   // clamped: every load stays in range, selects afterwards
        cb[u] = min(c, N - 1);
    }
    d4 acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = d4{0.0, 0.0, 0.0, 0.0};
    double a[2][4], b[2][4], an[2][4], bn[2][4];
    auto load = [&](int k0, double (&aa)[2][4], double (&bb)[2][4]) {
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int k = k0 + 4 * ks + lk;
            const int kc = min(k, K - 1);
            const bool pk = k < K;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const double x = A[ra[u] + lda * kc];
                const double y = Bm[kc + ldb * cb[u]];
                aa[u][ks] = (pk && pa[u]) ? x : 0.0;
                bb[u][ks] = (pk && pb[u]) ? y : 0.0;
            }
        }
    };
    load(0, a, b);
    for (int k0 = 0; k0 < K; k0 += 16) {
        const bool more = k0 + 16 < K;
        if (more) load(k0 + 16, an, bn);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v)
                    acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][ks], b[v][ks], acc[u][v], 0, 0, 0);
        if (more) {
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    a[u][ks] = an[u][ks];
                    b[u][ks] = bn[u][ks];
                }
        }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = i0 + 16 * u + 4 * r + lk, col = j0 + 16 * v + li;
                if (row < M && col < N) C[row + ldc * col] = acc[u][v][r];
            }
}

// Q_q(i, c) = sum_t v_t Y^{-1}(j_t, C_c) and Q'_q(i, c) = sum_t v_t X^(j_t, C_c) over
// the entries (i, j_t, v_t) of one row segment of A_q (rows of A_q in order, the
// entries of a row contiguous).  One wave per segment, lanes over c.  With slots
// the values are read from an E-vector (the dual residual G), block `qfix`; with
// seg_row == nullptr segment s is row s.
__global__ void __launch_bounds__(256)
k_cc_q(int64_t nseg, int n, int nc, const int *__restrict__ seg_q, const int *__restrict__ seg_row,
       const int64_t *__restrict__ seg_ptr, const int *__restrict__ seg_col, const double *__restrict__ seg_val,
       const int *__restrict__ seg_slot, const double *__restrict__ Mvec, int qfix, const double *__restrict__ YC,
       const double *__restrict__ XC, double *__restrict__ Q, double *__restrict__ Qp) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = int64_t(gridDim.x) * (blockDim.x >> 6);
    for (int64_t s = blockIdx.x * int64_t(blockDim.x >> 6) + (threadIdx.x >> 6); s < nseg; s += waves) {
        const int q = seg_q ? seg_q[s] : qfix;
        const int i = seg_row ? seg_row[s] : int(s);
        const int64_t t0 = seg_ptr[s], t1 = seg_ptr[s + 1];
        double *qb = Q + int64_t(q) * n * nc, *qpb = Qp + int64_t(q) * n * nc;
        for (int c = lane; c < nc; c += 64) {
            double sy = 0.0, sx = 0.0;
            for (int64_t t = t0; t < t1; ++t) {
                const int j = seg_col[t];
                const double v = seg_slot ? Mvec[seg_slot[t]] : seg_val[t];
                sy = fma(v, YC[c + int64_t(nc) * j], sy);
                sx = fma(v, XC[c + int64_t(nc) * j], sx);
            }
            qb[i + int64_t(n) * c] = sy;
            qpb[i + int64_t(n) * c] = sx;
        }
    }
}

// The same for |C| <= 16 with the lanes over the entries of the segment (long rows
// are not one serial chain): every lane keeps |C| partial sums of each product,
// reduced over the wave in a fixed order.
// Segments of at most kShortSeg entries go to k_cc_q16_short, one lane per segment
// over its entries in order (a wave per segment would idle most of its lanes and
// spend its time on the reductions); k_cc_q16 takes the longer ones.
constexpr int kShortSeg = 64;

__global__ void __launch_bounds__(256)
k_cc_q16_short(int64_t nseg, int n, int nc, const int *__restrict__ seg_q, const int *__restrict__ seg_row,
               const int64_t *__restrict__ seg_ptr, const int *__restrict__ seg_col,
               const double *__restrict__ seg_val, const int *__restrict__ seg_slot, const double *__restrict__ Mvec,
               int qfix, const double *__restrict__ YC, const double *__restrict__ XC, double *__restrict__ Q,
               double *__restrict__ Qp) {
    for (int64_t s = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; s < nseg; s += int64_t(gridDim.x) * blockDim.x) {
        const int64_t t0 = seg_ptr[s], t1 = seg_ptr[s + 1];
        if (t1 - t0 > kShortSeg) continue;   // k_cc_q16's
        const int q = seg_q ? seg_q[s] : qfix;
        const int i = seg_row ? seg_row[s] : int(s);
        double ay[16], ax[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) ay[c] = ax[c] = 0.0;
        for (int64_t t = t0; t < t1; ++t) {
            const int j = seg_col[t];
            const double v = seg_slot ? Mvec[seg_slot[t]] : seg_val[t];
            const double *yc = YC + int64_t(nc) * j, *xc = XC + int64_t(nc) * j;
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (c < nc) {
                    ay[c] = fma(v, yc[c], ay[c]);
                    ax[c] = fma(v, xc[c], ax[c]);
                }
        }
#pragma unroll
        for (int c = 0; c < 16; ++c)
            if (c < nc) {
                Q[int64_t(q) * n * nc + i + int64_t(n) * c] = ay[c];
                Qp[int64_t(q) * n * nc + i + int64_t(n) * c] = ax[c];
            }
    }
}

__global__ void __launch_bounds__(256)
k_cc_q16(int64_t nseg, int n, int nc, const int *__restrict__ seg_q, const int *__restrict__ seg_row,
         const int64_t *__restrict__ seg_ptr, const int *__restrict__ seg_col, const double *__restrict__ seg_val,
         const int *__restrict__ seg_slot, const double *__restrict__ Mvec, int qfix, const double *__restrict__ YC,
         const double *__restrict__ XC, double *__restrict__ Q, double *__restrict__ Qp) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = int64_t(gridDim.x) * (blockDim.x >> 6);
    for (int64_t s = blockIdx.x * int64_t(blockDim.x >> 6) + (threadIdx.x >> 6); s < nseg; s += waves) {
        const int64_t t0 = seg_ptr[s], t1 = seg_ptr[s + 1];
        if (t1 - t0 <= kShortSeg) continue;   // k_cc_q16_short's
        const int q = seg_q ? seg_q[s] : qfix;
        const int i = seg_row ? seg_row[s] : int(s);
        double ay[16], ax[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) ay[c] = ax[c] = 0.0;
        for (int64_t t = t0 + lane; t < t1; t += 64) {
            const int j = seg_col[t];
            const double v = seg_slot ? Mvec[seg_slot[t]] : seg_val[t];
            const double *yc = YC + int64_t(nc) * j, *xc = XC + int64_t(nc) * j;
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (c < nc) {
                    ay[c] = fma(v, yc[c], ay[c]);
                    ax[c] = fma(v, xc[c], ax[c]);
                }
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            if (c >= nc) break;
            double y = ay[c], x = ax[c];
            for (int o = 32; o > 0; o >>= 1) {
                y += __shfl_xor(y, o, 64);
                x += __shfl_xor(x, o, 64);
            }
            if (lane == 0) {
                Q[int64_t(q) * n * nc + i + int64_t(n) * c] = y;
                Qp[int64_t(q) * n * nc + i + int64_t(n) * c] = x;
            }
        }
    }
}

// H(a, i) = X^(ds_a, ds_i) Y^{-1}(ds_a, ds_i) on the diagonal support (nds x nds,
// column-major)
__global__ void __launch_bounds__(256)
k_had_ds(int n, int nds, const int *__restrict__ ds, const double *__restrict__ Xh, const double *__restrict__ Yi,
         double *__restrict__ H) {
    const int64_t total = int64_t(nds) * nds;
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < total; x += int64_t(gridDim.x) * blockDim.x) {
        const int a = int(x % nds);
        const int64_t i = x / nds;
        const int64_t src = ds[a] + int64_t(n) * ds[i];
        H[x] = Xh[src] * Yi[src];
    }
}

// diagT(a, q) = sum_i (X^ o Y^{-1})(ds_i, ds_a) D_q(ds_i) for the ndq constraints dq[] that
// have a diagonal part (when they are few; the other columns of diagT are zeroed
// beforehand): one wave per a reads column ds_a of X^ and Y^{-1} once (both are
// symmetric), its lanes' sums added in a fixed order
__global__ void __launch_bounds__(256)
k_diag_few(int n, int nds, const int *__restrict__ ds, const double *__restrict__ Xh, const double *__restrict__ Yi,
           const double *__restrict__ dmat, int ndq, const int *__restrict__ dq, double *__restrict__ diagT) {
    const int lane = threadIdx.x & 63;
    const int waves = gridDim.x * (blockDim.x >> 6);
    for (int a = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); a < nds; a += waves) {
        const int64_t ca = int64_t(n) * ds[a];
        double acc[kDqFew];
#pragma unroll
        for (int t = 0; t < kDqFew; ++t) acc[t] = 0.0;
        for (int i = lane; i < nds; i += 64) {
            const int64_t src = ds[i] + ca;
            const double hv = Xh[src] * Yi[src];
#pragma unroll
            for (int t = 0; t < kDqFew; ++t)
                if (t < ndq) acc[t] = fma(hv, dmat[i + int64_t(nds) * dq[t]], acc[t]);
        }
#pragma unroll
        for (int t = 0; t < kDqFew; ++t) {
            if (t >= ndq) break;
            double v = acc[t];
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) diagT[a + int64_t(nds) * dq[t]] = v;
        }
    }
}

// diagT(a, q) += sum_c P_q(ds_a, c) Y^{-1}(ds_a, C_c) + sum_c P'_q(ds_a, c) X^(ds_a, C_c)
// for q < nq (diagT: nds x nq column-major, already holding the D_q part)
__global__ void __launch_bounds__(256)
k_cc_diag(int n, int nc, int nds, int nq, const int *__restrict__ ds, const double *__restrict__ P,
          const double *__restrict__ Pp, const double *__restrict__ YC, const double *__restrict__ XC,
          double *__restrict__ diagT) {
    const int64_t total = int64_t(nds) * nq;
    for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < total; x += int64_t(gridDim.x) * blockDim.x) {
        const int ai = int(x % nds);
        const int q = int(x / nds);
        const int a = ds[ai];
        const double *pb = P + int64_t(q) * n * nc, *ppb = Pp + int64_t(q) * n * nc;
        double s = diagT[x];
        for (int c = 0; c < nc; ++c) {
            s = fma(pb[a + int64_t(n) * c], YC[c + int64_t(nc) * a], s);
            s = fma(ppb[a + int64_t(n) * c], XC[c + int64_t(nc) * a], s);
        }
        diagT[x] = s;
    }
}

// the dual residual's column of diagT: (X^ G Y^{-1})(ds_a, ds_a) = sum_j Z(ds_a, j) Y^{-1}(ds_a, j)
// with Z = X^ G column-major; one wave per diagonal position
__global__ void __launch_bounds__(256)
k_cc_diag_g(int n, int nds, const int *__restrict__ ds, const double *__restrict__ Z, const double *__restrict__ Yi,
            double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = int64_t(gridDim.x) * (blockDim.x >> 6);
    for (int64_t ai = blockIdx.x * int64_t(blockDim.x >> 6) + (threadIdx.x >> 6); ai < nds; ai += waves) {
        const int a = ds[ai];
        double s = 0.0;
        for (int j = lane; j < n; j += 64) s = fma(Z[a + int64_t(n) * j], Yi[a + int64_t(n) * j], s);
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) out[ai] = s;
    }
}

// B(p, q) = <P_p, Q_q> + <P'_p, Q'_q> + sum_a Dm(a, p) diagT(a, q) for p >= max(q, pmin)
// (q = the column of this workgroup's pair), a fixed-order reduction per pair.  One
// workgroup per output entry of the listed columns; out(p, q) at out[p + ldo * (q - q0)].
__global__ void __launch_bounds__(256)
k_cc_b(int m, int64_t len, int nds, int q0, int nqcols, const double *__restrict__ P, const double *__restrict__ Pp,
       const double *__restrict__ Q, const double *__restrict__ Qp, const double *__restrict__ Dm,
       const double *__restrict__ diagT, int lower, double *__restrict__ out, int64_t ldo) {
    __shared__ double red[4];
    const int64_t npairs = int64_t(m) * nqcols;
    for (int64_t x = blockIdx.x; x < npairs; x += gridDim.x) {
        const int p = int(x % m);
        const int q = q0 + int(x / m);
        if (lower && p < q) continue;   // uniform over the workgroup
        const double *pp = P + int64_t(p) * len, *ppp = Pp + int64_t(p) * len;
        const double *qq = Q + int64_t(q) * len, *qqp = Qp + int64_t(q) * len;
        double s = 0.0;
        for (int64_t k = threadIdx.x; k < len; k += blockDim.x) s = fma(pp[k], qq[k], fma(ppp[k], qqp[k], s));
        for (int a = threadIdx.x; a < nds; a += blockDim.x)
            s = fma(Dm[a + int64_t(nds) * p], diagT[a + int64_t(nds) * q], s);
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) out[p + ldo * (q - q0)] = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
    }
}

__global__ void k_zero(int64_t len, double *__restrict__ x) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < len; i += int64_t(gridDim.x) * blockDim.x)
        x[i] = 0.0;
}

int grid_for(int64_t items, int per) {
    int64_t g = (items + per - 1) / per;
    if (g < 1) g = 1;
    if (g > 16384) g = 16384;
    return int(g);
}

}  // namespace

size_t cc_work_doubles(const DevStruct &d) {
    const size_t blk = size_t(d.n) * d.nc;
    // P, P' (m blocks), Q, Q' (m + 1 blocks: the last for G), Y^{-1}(C, :), X^(C, :),
    // diagT (nds x (m + 1))
    return 2 * blk * d.m + 2 * blk * (d.m + 1) + 2 * size_t(d.nc) * d.n + size_t(d.nds) * (d.m + 1);
}

namespace {

struct CcWork {
    double *P, *Pp, *Q, *Qp, *YC, *XC, *diagT;
};

CcWork cc_split(const DevStruct &d, double *work) {
    const size_t blk = size_t(d.n) * d.nc;
    CcWork w;
    w.P = work;
    w.Pp = w.P + blk * d.m;
    w.Q = w.Pp + blk * d.m;
    w.Qp = w.Q + blk * (d.m + 1);
    w.YC = w.Qp + blk * (d.m + 1);
    w.XC = w.YC + size_t(d.nc) * d.n;
    w.diagT = w.XC + size_t(d.nc) * d.n;
    return w;
}

}  // namespace

void launch_scm_cc(const DevStruct &d, const double *Xh, const double *Yi, double *H, double *work, double *B,
                   int64_t ldb, hipStream_t st) {
    const int n = d.n, m = d.m, nc = d.nc, nds = d.nds;
    CcWork w = cc_split(d, work);
    const int64_t blk = int64_t(n) * nc;
    if (nc > 0) {
        hipLaunchKernelGGL(k_gather_rows, dim3(grid_for(int64_t(nc) * n, 256)), dim3(256), 0, st, n, nc, d.ccol, Yi,
                           Xh, w.YC, w.XC);
        // P = X^ U_cat, P' = Y^{-1} U_cat
        hipLaunchKernelGGL(k_gemm_nn, dim3((n + 63) / 64, (m * nc + 63) / 64, 2), dim3(256), 0, st, n, m * nc, n, Xh,
                           Yi, int64_t(n), d.ucat, int64_t(n), w.P, w.Pp, int64_t(n));
        hipLaunchKernelGGL(k_zero, dim3(grid_for(2 * blk * (m + 1), 256)), dim3(256), 0, st, 2 * blk * (m + 1), w.Q);
        if (nc <= 16)
            hipLaunchKernelGGL(k_cc_q16_short, dim3(grid_for(d.nseg, 256)), dim3(256), 0, st, d.nseg, n, nc, d.seg_q,
                               d.seg_row, d.seg_ptr, d.seg_col, d.seg_val, (const int *)nullptr,
                               (const double *)nullptr, 0, w.YC, w.XC, w.Q, w.Qp);
        hipLaunchKernelGGL(nc <= 16 ? k_cc_q16 : k_cc_q, dim3(grid_for(d.nseg, 4)), dim3(256), 0, st, d.nseg, n, nc,
                           d.seg_q, d.seg_row, d.seg_ptr, d.seg_col, d.seg_val, (const int *)nullptr,
                           (const double *)nullptr, 0, w.YC, w.XC, w.Q, w.Qp);
    }
    if (nds > 0) {
        // diagT(., q) = (X^ o Y^{-1})(Ds, Ds) D_q, then the U_q terms; with few D_q
        // nonzero, one pass over the columns Ds of X^ and Y^{-1} instead of the product
        if (d.ndq >= 0) {
            hipLaunchKernelGGL(k_zero, dim3(grid_for(int64_t(nds) * m, 256)), dim3(256), 0, st, int64_t(nds) * m,
                               w.diagT);
            if (d.ndq > 0)
                hipLaunchKernelGGL(k_diag_few, dim3(grid_for(nds, 4)), dim3(256), 0, st, n, nds, d.ds, Xh, Yi,
                                   d.dmat, d.ndq, d.dq, w.diagT);
        } else {
            hipLaunchKernelGGL(k_had_ds, dim3(grid_for(int64_t(nds) * nds, 256)), dim3(256), 0, st, n, nds, d.ds, Xh,
                               Yi, H);
            hipLaunchKernelGGL(k_gemm_nn, dim3((nds + 63) / 64, (m + 63) / 64, 1), dim3(256), 0, st, nds, m, nds, H,
                               H, int64_t(nds), d.dmat, int64_t(nds), w.diagT, w.diagT, int64_t(nds));
        }
        if (nc > 0)
            hipLaunchKernelGGL(k_cc_diag, dim3(grid_for(int64_t(nds) * m, 256)), dim3(256), 0, st, n, nc, nds, m, d.ds,
                               w.P, w.Pp, w.YC, w.XC, w.diagT);
    }
    hipLaunchKernelGGL(k_cc_b, dim3(grid_for(int64_t(m) * m, 1)), dim3(256), 0, st, m, blk, nds, 0, m, w.P, w.Pp,
                       w.Q, w.Qp, d.dmat, w.diagT, 1, B, ldb);
}

void launch_scm_cc_extra_column(const DevStruct &d, const double *Mvec, const double *Xh, const double *Yi,
                                double *Z, double *work, double *col, hipStream_t st) {
    // the blocks P, P' and the rows Y^{-1}(C, :), X^(C, :) of the same X^ and Y^{-1}
    // are those left by launch_scm_cc
    const int n = d.n, m = d.m, nc = d.nc, nds = d.nds;
    CcWork w = cc_split(d, work);
    const int64_t blk = int64_t(n) * nc;
    if (nc > 0) {
        hipLaunchKernelGGL(k_zero, dim3(grid_for(blk, 256)), dim3(256), 0, st, blk, w.Q + blk * m);
        hipLaunchKernelGGL(k_zero, dim3(grid_for(blk, 256)), dim3(256), 0, st, blk, w.Qp + blk * m);
        // rows of G: by symmetry, column j of the aggregate pattern lists the entries of row j
        if (nc <= 16)
            hipLaunchKernelGGL(k_cc_q16_short, dim3(grid_for(n, 256)), dim3(256), 0, st, int64_t(n), n, nc,
                               (const int *)nullptr, (const int *)nullptr, d.ag_cptr, d.ag_row,
                               (const double *)nullptr, d.ag_slot, Mvec, m, w.YC, w.XC, w.Q, w.Qp);
        hipLaunchKernelGGL(nc <= 16 ? k_cc_q16 : k_cc_q, dim3(grid_for(n, 4)), dim3(256), 0, st, int64_t(n), n, nc,
                           (const int *)nullptr, (const int *)nullptr, d.ag_cptr, d.ag_row, (const double *)nullptr,
                           d.ag_slot, Mvec, m, w.YC, w.XC, w.Q, w.Qp);
    }
    if (nds > 0) {
        launch_zcol(d, Xh, Mvec, Z, st);
        hipLaunchKernelGGL(k_cc_diag_g, dim3(grid_for(nds, 4)), dim3(256), 0, st, n, nds, d.ds, Z, Yi,
                           w.diagT + int64_t(nds) * m);
    }
    hipLaunchKernelGGL(k_cc_b, dim3(grid_for(m, 1)), dim3(256), 0, st, m, blk, nds, m, 1, w.P, w.Pp, w.Q, w.Qp,
                       d.dmat, w.diagT, 0, col, int64_t(m));
}

}  // namespace sdpc
