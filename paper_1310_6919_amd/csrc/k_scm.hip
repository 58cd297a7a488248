// Schur complement matrix (eq. SCM, evaluated through the dense columns of
// X^ and Y^{-1} as in eq. newSCM2), the right-hand side of the SCE and the
// primal direction on E (eq. newdX2).
//
//  hadamard   every A_k (k >= 1) is a single diagonal entry v_k e_{a_k}
//             e_{a_k}^T (the max-cut form): B_pq = v_p v_q X^(a_p,a_q)
//             Y^{-1}(a_q,a_p).
//  general    for each q: W = X^ A_q restricted to the nonzero columns K_q
//             of A_q (row-major), T_q(a, b) = W(a, :) . Y^{-1}(K_q, b) on the
//             union support of A_1..A_m, then B_pq = sum over supp A_p of
//             [A_p]_ab T_q(a, b).  The same three steps with A_q replaced by
//             the dual residual G give A_p . (X^ G Y^{-1}) for the SCE
//             right-hand side.
//  dX         dX = beta mu Y^{-1} - Xbar - (X^ dY Y^{-1} + Y^{-1} dY X^)/2 on
//             the slots of E only (eq. newdX2 and the symmetrisation of
//             eq. dX), with W = X^ dY.
#include "kernels.h"

namespace sdpc {

namespace {

__global__ void __launch_bounds__(256)
k_scm_had(int m, int n, const int *__restrict__ pos, const double *__restrict__ val,
          const double *__restrict__ Xh, const double *__restrict__ Yi, double *__restrict__ B, int64_t ldb) {
    const int q = blockIdx.y;
    const int c = pos[q];
    const double vq = val[q];
    const double *xc = Xh + int64_t(n) * c;
    const double *yc = Yi + int64_t(n) * c;
    for (int p = q + blockIdx.x * blockDim.x + threadIdx.x; p < m; p += gridDim.x * blockDim.x) {
        const int a = pos[p];
        B[p + ldb * q] = val[p] * vq * xc[a] * yc[a];
    }
}

// W(a, j) = sum over entries t of column j: value_t * X^(row_t, a); row-major, K columns
__global__ void __launch_bounds__(256)
k_dense_times_sparse(int n, int K, const int64_t *__restrict__ cptr, const int *__restrict__ rows,
                     const double *__restrict__ vals, const int *__restrict__ slots,
                     const double *__restrict__ Mvec, const double *__restrict__ Xh, double *__restrict__ W) {
    for (int a = blockIdx.x; a < n; a += gridDim.x) {
        const double *xa = Xh + int64_t(n) * a;   // column a of X^ = row a (symmetric)
        double *wa = W + int64_t(K) * a;
        for (int j = threadIdx.x; j < K; j += blockDim.x) {
            double s = 0.0;
            for (int64_t t = cptr[j]; t < cptr[j + 1]; ++t) {
                const double v = slots ? Mvec[slots[t]] : vals[t];
                s += v * xa[rows[t]];
            }
            wa[j] = s;
        }
    }
}

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// T(s) = W(a, :) . Y^{-1}(kcol, S_col[s]) for the support entries s of row a
__global__ void __launch_bounds__(256)
k_support_dots(int n, int K, const int *__restrict__ kcol, const int64_t *__restrict__ S_rowptr,
               const int *__restrict__ S_col, const double *__restrict__ W, const double *__restrict__ Yi,
               double *__restrict__ T) {
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
    for (int a = blockIdx.x; a < n; a += gridDim.x) {
        const double *wa = W + int64_t(K) * a;
        for (int64_t s = S_rowptr[a] + wv; s < S_rowptr[a + 1]; s += 4) {
            const double *yb = Yi + int64_t(n) * S_col[s];
            double acc = 0.0;
            if (kcol) {
                for (int j = lane; j < K; j += 64) acc += wa[j] * yb[kcol[j]];
            } else {
                for (int j = lane; j < K; j += 64) acc += wa[j] * yb[j];
            }
            acc = wave_sum(acc);
            if (lane == 0) T[s] = acc;
        }
    }
}

__global__ void __launch_bounds__(256)
k_contract(int m, int q0, const int64_t *__restrict__ am_ptr, const int64_t *__restrict__ am_sidx,
           const double *__restrict__ am_val, const double *__restrict__ T, double *__restrict__ out) {
    for (int p = q0 + blockIdx.x * blockDim.x + threadIdx.x; p < m; p += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int64_t t = am_ptr[p]; t < am_ptr[p + 1]; ++t) s += am_val[t] * T[am_sidx[t]];
        out[p] = s;
    }
}

// g_p = b_p - beta mu A_p . Y^{-1} + h_p: one wave per constraint, its entries split
// over the lanes and summed in a fixed order
__global__ void __launch_bounds__(256)
k_rhs(int m, int n, const int64_t *__restrict__ con_ptr, const int *__restrict__ con_pi,
      const int *__restrict__ con_pj, const double *__restrict__ con_val, const double *__restrict__ b,
      const double *__restrict__ Yi, const double *__restrict__ hcol, double beta_mu, double *__restrict__ g) {
    const int lane = threadIdx.x & 63;
    const int waves = gridDim.x * (blockDim.x >> 6);
    for (int p = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); p < m; p += waves) {
        double ay = 0.0;
        for (int64_t t = con_ptr[p + 1] + lane; t < con_ptr[p + 2]; t += 64)
            ay = fma(con_val[t], Yi[con_pi[t] + int64_t(n) * con_pj[t]], ay);
        for (int o = 32; o > 0; o >>= 1) ay += __shfl_xor(ay, o, 64);
        if (lane == 0) g[p] = b[p] - beta_mu * ay + hcol[p];
    }
}

__global__ void __launch_bounds__(256)
k_dX(int64_t nslot, int n, const int *__restrict__ slot_row, const int *__restrict__ slot_col,
     const double *__restrict__ W, const double *__restrict__ Yi, const double *__restrict__ Xbar,
     double beta_mu, double *__restrict__ dX) {
    const int lane = threadIdx.x % 64;
    const int64_t waves = int64_t(gridDim.x) * 4;
    for (int64_t s = blockIdx.x * 4 + threadIdx.x / 64; s < nslot; s += waves) {
        const int i = slot_row[s];
        if (i < 0) {
            if (lane == 0) dX[s] = 0.0;
            continue;
        }
        const int j = slot_col[s];
        const double *wi = W + int64_t(n) * i, *wj = W + int64_t(n) * j;
        const double *yi = Yi + int64_t(n) * i, *yj = Yi + int64_t(n) * j;
        double acc = 0.0;
        for (int d = lane; d < n; d += 64) acc += wi[d] * yj[d] + wj[d] * yi[d];
        acc = wave_sum(acc);
        if (lane == 0) dX[s] = beta_mu * yj[i] - Xbar[s] - 0.5 * acc;
    }
}

typedef double d4 __attribute__((ext_vector_type(4)));   // one MFMA accumulator

// The same two products for a group of 32 columns whose rows form the union U:
// Z(P, G) = X^(P, U) M(U, G) is a dense product on the FP64 MFMA, with M(U, G)
// gathered into LDS kZmRows rows at a time.  It is formed transposed, Z^T = M^T X^T (lane l
// supplies A(l % 16, l / 16) and B(l / 16, l % 16); element r of the result is
// C(4 r + l / 16, l % 16)), so 16 lanes hold 16 consecutive rows p of one column:
// coalesced reads of X^ and Y^{-1} and writes of Z.  Each workgroup takes 64 rows
// (16 per wave).  RHS: the partial sums over the group's columns of
// (X^ M)(p, c) Y^{-1}(p, c), whose total is h_p = (X^ M Y^{-1})(p, p) in the max-cut
// form; otherwise Z is stored.
template <bool RHS>
__global__ void __launch_bounds__(256)
k_zm_mma(int n, const int *__restrict__ groups, const int64_t *__restrict__ zg_ptr, const int *__restrict__ zg_rows,
         const int *__restrict__ zg_slot, const int *__restrict__ zg_col, const int *__restrict__ zg_piece,
         const double *__restrict__ Mvec, const double *__restrict__ Xh, const double *__restrict__ Yi,
         double *__restrict__ out, double *__restrict__ zpart) {
    __shared__ double Mb[kZmRows * 33];
    __shared__ int Ur[kZmRows];
    const int vg = groups[blockIdx.y];   // a group or a piece of one
    const int g = zg_col[vg];            // its columns 32 g ..
    const int64_t u0 = zg_ptr[vg];
    const int K = int(zg_ptr[vg + 1] - u0);   // a multiple of 4
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    const int p = 64 * blockIdx.x + 16 * wv + li;
    const int pc = min(p, n - 1);   // clamped: loads stay in range
    d4 acc[2];
    acc[0] = acc[1] = d4{0.0, 0.0, 0.0, 0.0};
    // the union rows in chunks of kZmRows, each chunk of M(U, G) staged in LDS
    for (int kb = 0; kb < K; kb += kZmRows) {
        const int KK = min(kZmRows, K - kb);
        __syncthreads();   // the previous chunk has been consumed
        for (int idx = threadIdx.x; idx < KK * 32; idx += blockDim.x) {
            const int sl = zg_slot[32 * (u0 + kb) + idx];
            Mb[(idx / 32) * 33 + idx % 32] = (sl >= 0) ? Mvec[sl] : 0.0;
        }
        for (int k = threadIdx.x; k < KK; k += blockDim.x) Ur[k] = zg_rows[u0 + kb + k];
        __syncthreads();
#pragma unroll 4
        for (int ks = 0; ks < KK / 4; ++ks) {
            const int k = 4 * ks + lk;
            const double x = Xh[pc + int64_t(n) * Ur[k]];
            acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(Mb[k * 33 + li], x, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(Mb[k * 33 + 16 + li], x, acc[1], 0, 0, 0);
        }
    }
    if (RHS) {
        double sacc = 0.0;
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = 32 * g + 16 * t + 4 * r + lk;
                const double y = Yi[pc + int64_t(n) * min(c, n - 1)];
                sacc += (c < n) ? acc[t][r] * y : 0.0;
            }
        sacc += __shfl_xor(sacc, 16);
        sacc += __shfl_xor(sacc, 32);
        if (lk == 0 && p < n) out[int64_t(vg) * n + p] = sacc;
    } else {
        const int piece = zg_piece[vg];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = 32 * g + 16 * t + 4 * r + lk;
                if (p < n && c < n) {
                    if (piece < 0)
                        out[p + int64_t(n) * c] = acc[t][r];
                    else
                        zpart[(int64_t(piece) * 32 + (c - 32 * g)) * n + p] = acc[t][r];
                }
            }
    }
}

// Z(p, 32 g + cc) = the sum of the pieces' products in piece order, for the column
// groups that were cut (blockIdx.y) and their columns cc (blockIdx.z)
__global__ void __launch_bounds__(256)
k_zm_reduce(int n, const int *__restrict__ zs_g, const int *__restrict__ zs_ptr, const double *__restrict__ zpart,
            double *__restrict__ Z) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int cc = blockIdx.z, c = 32 * zs_g[blockIdx.y] + cc;
    if (p >= n || c >= n) return;
    double s = 0.0;
    for (int q = zs_ptr[blockIdx.y]; q < zs_ptr[blockIdx.y + 1]; ++q) s += zpart[(int64_t(q) * 32 + cc) * n + p];
    Z[p + int64_t(n) * c] = s;
}

// out[k] = sum over the parts of part[c n + pos[k]] (pos maps constraint k to its
// position; null: the identity): 64 outputs per workgroup, each wave a quarter of
// the parts, the four partial sums added in a fixed order
__global__ void __launch_bounds__(256)
k_sum_partials(int n, int nparts, const double *__restrict__ part, const int *__restrict__ pos,
               double *__restrict__ out) {
    __shared__ double ps[4][64];
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int k = blockIdx.x * 64 + l;
    double s = 0.0;
    if (k < n) {
        const int p = pos ? pos[k] : k;
        for (int c = wv; c < nparts; c += 4) s += part[int64_t(c) * n + p];
    }
    ps[wv][l] = s;
    __syncthreads();
    if (wv == 0 && k < n) out[k] = (ps[0][l] + ps[1][l]) + (ps[2][l] + ps[3][l]);
}

// dX on E, block-tiled: for storage block b and a chunk of 256 values of d, partial
// sums of T(R_b, cols_b) = Z(R_b, :) Y^{-1}(:, cols_b) and T(cols_b, R_b)^T =
// Y^{-1}(R_b, :) Z(cols_b, :)^T with T = X^ dY Y^{-1} (Z = X^ dY column-major; Y^{-1} is
// symmetric, so both products read rows of column-major matrices: coalesced).  part
// holds [chunk][2][nslot].  On the FP64 MFMA (16 x 16 x 4; lane l supplies A(l % 16,
// l / 16) and B(l / 16, l % 16), element r of the result is C(4 r + l / 16, l % 16)):
// wave w owns the 16-row tiles w, w + 4, ... of the panel and both 16-column tiles.
constexpr int kDxChunk = 256;

__global__ void __launch_bounds__(256)
k_dX_mma(int n, int nslot_i, const int *__restrict__ bl_first, const int64_t *__restrict__ bl_rptr,
         const int *__restrict__ bl_rows, const int64_t *__restrict__ bl_off, const double *__restrict__ Z,
         const double *__restrict__ Yi, double *__restrict__ part) {
    const int b = blockIdx.x, ch = blockIdx.y;
    const int F = bl_first[b], w = bl_first[b + 1] - F;
    const int64_t r0 = bl_rptr[b];
    const int h = int(bl_rptr[b + 1] - r0);
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    const int c0 = min(F + li, n - 1), c1 = min(F + 16 + li, n - 1);   // clamped: loads stay in range
    const bool pc0 = li < w, pc1 = 16 + li < w;
    const int d_begin = ch * kDxChunk;
    double *p1 = part + int64_t(ch) * 2 * nslot_i;
    double *p2 = p1 + nslot_i;
    const int64_t off = bl_off[b];
    for (int rt = wv; 16 * rt < h; rt += 4) {   // 16-row tiles of the panel
        const int p = 16 * rt + li;             // panel row supplied by this lane
        const int row = bl_rows[r0 + min(p, h - 1)];
        const bool prow = p < h;
        d4 o1[2], o2[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) o1[t] = o2[t] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int ks = 0; ks < kDxChunk / 4; ++ks) {
            const int dd = d_begin + 4 * ks + lk;
            const bool pd = dd < n;
            const int64_t cd = int64_t(n) * min(dd, n - 1);
            const double za = Z[row + cd], ya = Yi[row + cd];
            const double y0 = Yi[c0 + cd], y1 = Yi[c1 + cd], z0 = Z[c0 + cd], z1 = Z[c1 + cd];
            const double a1 = (prow && pd) ? za : 0.0, a2 = (prow && pd) ? ya : 0.0;
            o1[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, (pc0 && pd) ? y0 : 0.0, o1[0], 0, 0, 0);
            o1[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, (pc1 && pd) ? y1 : 0.0, o1[1], 0, 0, 0);
            o2[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, (pc0 && pd) ? z0 : 0.0, o2[0], 0, 0, 0);
            o2[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, (pc1 && pd) ? z1 : 0.0, o2[1], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int pr = 16 * rt + 4 * r + lk, c = 16 * t + li;
                if (pr < h && c < w) {
                    const int64_t sl = off + pr + int64_t(h) * c;
                    p1[sl] = o1[t][r];
                    p2[sl] = o2[t][r];
                }
            }
    }
}

__global__ void __launch_bounds__(256)
k_dX_finish(int64_t nslot, int n, int nch, const int *__restrict__ slot_row, const int *__restrict__ slot_col,
            const double *__restrict__ part, const double *__restrict__ Yi, const double *__restrict__ Xbar,
            double beta_mu, double *__restrict__ dX) {
    for (int64_t s = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; s < nslot; s += int64_t(gridDim.x) * blockDim.x) {
        const int i = slot_row[s];
        if (i < 0) {
            dX[s] = 0.0;
            continue;
        }
        const int j = slot_col[s];
        double t = 0.0;
        for (int c = 0; c < nch; ++c) t += part[(2 * c) * nslot + s] + part[(2 * c + 1) * nslot + s];
        dX[s] = beta_mu * Yi[i + int64_t(n) * j] - Xbar[s] - 0.5 * t;
    }
}

__global__ void k_fill(int len, double v, double *__restrict__ x) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x) x[i] = v;
}

int grid_cap(int64_t items, int per) {
    int64_t g = (items + per - 1) / per;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return int(g);
}

}  // namespace

void launch_scm_hadamard(const DevStruct &d, const double *Xh, const double *Yi, double *B, int64_t ldb,
                         hipStream_t st) {
    const int gx = grid_cap(d.m, 256) > 16 ? 16 : grid_cap(d.m, 256);
    hipLaunchKernelGGL(k_scm_had, dim3(gx, d.m), dim3(256), 0, st, d.m, d.n, d.had_pos, d.had_val, Xh, Yi, B, ldb);
}

void launch_dense_times_agg(const DevStruct &d, const double *Xh, const double *Mvec, double *W, hipStream_t st) {
    hipLaunchKernelGGL(k_dense_times_sparse, dim3(grid_cap(d.n, 1)), dim3(256), 0, st, d.n, d.n, d.ag_cptr,
                       d.ag_row, (const double *)nullptr, d.ag_slot, Mvec, Xh, W);
}

void launch_scm_extra_column(const DevStruct &d, const double *Mvec, const double *Xh, const double *Yi, double *W,
                             double *T, double *col, hipStream_t st) {
    // W = X^ M over all n columns of the aggregate pattern, then the support dots and the contraction
    hipLaunchKernelGGL(k_dense_times_sparse, dim3(grid_cap(d.n, 1)), dim3(256), 0, st, d.n, d.n, d.ag_cptr,
                       d.ag_row, (const double *)nullptr, d.ag_slot, Mvec, Xh, W);
    hipLaunchKernelGGL(k_support_dots, dim3(grid_cap(d.n, 1)), dim3(256), 0, st, d.n, d.n, (const int *)nullptr,
                       d.S_rowptr, d.S_col, W, Yi, T);
    hipLaunchKernelGGL(k_contract, dim3(grid_cap(d.m, 256)), dim3(256), 0, st, d.m, 0, d.am_ptr, d.am_sidx,
                       d.am_val, T, col);
}

void launch_scm_general(const DevStruct &d, const int64_t *kq_ptr_host, const double *Xh, const double *Yi,
                        double *W, double *T, double *B, int64_t ldb, hipStream_t st) {
    for (int q = 0; q < d.m; ++q) {
        const int64_t c0 = kq_ptr_host[q];
        const int K = int(kq_ptr_host[q + 1] - c0);
        if (K == 0) {
            hipLaunchKernelGGL(k_fill, dim3(grid_cap(d.m - q, 256)), dim3(256), 0, st, d.m - q, 0.0,
                               B + ldb * q + q);
            continue;
        }
        hipLaunchKernelGGL(k_dense_times_sparse, dim3(grid_cap(d.n, 1)), dim3(256), 0, st, d.n, K,
                           d.aq_cptr + c0, d.aq_row, d.aq_val, (const int *)nullptr, (const double *)nullptr, Xh,
                           W);
        hipLaunchKernelGGL(k_support_dots, dim3(grid_cap(d.n, 1)), dim3(256), 0, st, d.n, K, d.kq_col + c0,
                           d.S_rowptr, d.S_col, W, Yi, T);
        hipLaunchKernelGGL(k_contract, dim3(grid_cap(d.m - q, 256)), dim3(256), 0, st, d.m, q, d.am_ptr,
                           d.am_sidx, d.am_val, T, B + ldb * q);
    }
}

void launch_zcol(const DevStruct &d, const double *Xh, const double *Mvec, double *Z, hipStream_t st) {
    if (d.nzg_mma > 0)
        hipLaunchKernelGGL(k_zm_mma<false>, dim3((d.n + 63) / 64, d.nzg_mma), dim3(256), 0, st, d.n, d.zg_mma,
                           d.zg_ptr, d.zg_rows, d.zg_slot, d.zg_col, d.zg_piece, Mvec, Xh, (const double *)nullptr,
                           Z, d.zpart);
    if (d.nzsplit > 0)
        hipLaunchKernelGGL(k_zm_reduce, dim3((d.n + 255) / 256, d.nzsplit, 32), dim3(256), 0, st, d.n, d.zs_g, d.zs_ptr,
                           (const double *)d.zpart, Z);
}

int rhs_had_parts(const DevStruct &d) { return d.nzg; }

void launch_rhs_hadamard(const DevStruct &d, const double *Mvec, const double *Xh, const double *Yi, double *part,
                         double *hcol, hipStream_t st) {
    const int nparts = rhs_had_parts(d);
    if (d.nzg_mma > 0)
        hipLaunchKernelGGL(k_zm_mma<true>, dim3((d.n + 63) / 64, d.nzg_mma), dim3(256), 0, st, d.n, d.zg_mma,
                           d.zg_ptr, d.zg_rows, d.zg_slot, d.zg_col, d.zg_piece, Mvec, Xh, Yi, part,
                           (double *)nullptr);
    hipLaunchKernelGGL(k_sum_partials, dim3((d.m + 63) / 64), dim3(256), 0, st, d.m, nparts,
                       (const double *)part, d.had_pos, hcol);
}

int dX_chunks(const DevStruct &d) { return (d.n + kDxChunk - 1) / kDxChunk; }

void launch_dX_blocked(const DevStruct &d, const double *Z, const double *Yi, const double *Xbar, double beta_mu,
                       double *part, double *dX, hipStream_t st) {
    const int nch = dX_chunks(d);
    hipLaunchKernelGGL(k_dX_mma, dim3(d.nb, nch), dim3(256), 0, st, d.n, int(d.nslot), d.bl_first, d.bl_rptr,
                       d.bl_rows, d.bl_off, Z, Yi, part);
    hipLaunchKernelGGL(k_dX_finish, dim3(grid_cap(d.nslot, 256)), dim3(256), 0, st, d.nslot, d.n, nch, d.slot_row,
                       d.slot_col, (const double *)part, Yi, Xbar, beta_mu, dX);
}

void launch_rhs(const DevStruct &d, const double *Yi, const double *h, double beta_mu, double *g, double *work,
                hipStream_t st) {
    if (launch_con_chunks(d, true, Yi, beta_mu, h, g, work, st)) return;
    hipLaunchKernelGGL(k_rhs, dim3(grid_cap(d.m, 4)), dim3(256), 0, st, d.m, d.n, d.con_ptr, d.con_pi, d.con_pj,
                       d.con_val, d.b, Yi, h, beta_mu, g);
}

void launch_dX(const DevStruct &d, const double *W, const double *Yi, const double *Xbar, double beta_mu, double *dX,
               hipStream_t st) {
    hipLaunchKernelGGL(k_dX, dim3(grid_cap(d.nslot, 4)), dim3(256), 0, st, d.nslot, d.n, d.slot_row, d.slot_col, W,
                       Yi, Xbar, beta_mu, dX);
}

}  // namespace sdpc
