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

__global__ void __launch_bounds__(256)
k_rhs(int m, int n, const int64_t *__restrict__ con_ptr, const int *__restrict__ con_pi,
      const int *__restrict__ con_pj, const double *__restrict__ con_val, const double *__restrict__ b,
      const double *__restrict__ Yi, const double *__restrict__ hcol, double beta_mu, double *__restrict__ g) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < m; p += gridDim.x * blockDim.x) {
        double ay = 0.0;
        for (int64_t t = con_ptr[p + 1]; t < con_ptr[p + 2]; ++t)
            ay += con_val[t] * Yi[con_pi[t] + int64_t(n) * con_pj[t]];
        g[p] = b[p] - beta_mu * ay + hcol[p];
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

void launch_rhs(const DevStruct &d, const double *Yi, const double *h, double beta_mu, double *g, hipStream_t st) {
    hipLaunchKernelGGL(k_rhs, dim3(grid_cap(d.m, 256)), dim3(256), 0, st, d.m, d.n, d.con_ptr, d.con_pi, d.con_pj,
                       d.con_val, d.b, Yi, h, beta_mu, g);
}

void launch_dX(const DevStruct &d, const double *W, const double *Yi, const double *Xbar, double beta_mu, double *dX,
               hipStream_t st) {
    hipLaunchKernelGGL(k_dX, dim3(grid_cap(d.nslot, 4)), dim3(256), 0, st, d.nslot, d.n, d.slot_row, d.slot_col, W,
                       Yi, Xbar, beta_mu, dX);
}

}  // namespace sdpc
