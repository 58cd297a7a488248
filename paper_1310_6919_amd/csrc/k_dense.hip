// Dense FP64 Cholesky of the Schur complement matrix, B = R R^T (type (i) of
// Section 3.1), and the two triangular solves of the SCE (eq. SCE).
//
// Right-looking blocked algorithm with 64-wide block columns:
//   k_potrf_diag   one workgroup factorises the 64 x 64 diagonal block in LDS
//                  and forms the inverse of its factor at the same time
//                  (forward elimination against the identity, one column per
//                  pivot step);
//   k_trsm_panel   R(I, J) = B(I, J) R(J, J)^{-T} for every 64-row tile below,
//                  as a product with the explicit inverse;
//   k_syrk_tiles   B(I, K) -= R(I, J) R(K, J)^T for every lower tile pair of the
//                  trailing matrix.
// Rows beyond m can ride along: with the right-hand side g stored as row m,
// the same sweep leaves R^{-1} g in that row (the forward substitution of the
// SCE for free), and only the backward substitution R^T x = R^{-1} g remains.
// Both products run on the FP64 matrix cores (v_mfma_f64_16x16x4f64): each
// of the four waves of a workgroup owns a 32 x 32 quadrant of the 64 x 64
// output tile, i.e. 2 x 2 MFMA blocks of 16 x 16.
#include "chol_reg.h"
#include "kernels.h"

namespace sdpc {

namespace {

constexpr int NB = 64;
constexpr int LDT = NB + 1;   // padded LDS row length

typedef double d4 __attribute__((ext_vector_type(4)));

// C(64x64) = A(64xK) * Bm(64xK)^T from LDS (row-major, ld LDT), K <= 64.
// Result returned per wave as acc[2][2] (16x16 blocks of its 32x32 quadrant).
// Operand layout of the FP64 16x16x4 MFMA: lane l supplies A(l % 16, l / 16)
// and B(l / 16, l % 16); element r of lane l's result is D(4 r + l / 16, l % 16)
// (checked on gfx950 with a lane-layout probe).
// Here: lane l, element r holds C(qr + 16 ti + 4 r + l / 16, qc + 16 tj + l % 16).
__device__ inline void tile_gemm_nt(const double *A, const double *Bm, int K, d4 acc[2][2]) {
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    const int qr = 32 * (w % 2), qc = 32 * (w / 2);
    const int li = lane % 16, lk = lane / 16;
    for (int ti = 0; ti < 2; ++ti)
        for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = d4{0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < K; k += 4) {
        double a[2], b[2];
        for (int t = 0; t < 2; ++t) {
            a[t] = A[(qr + 16 * t + li) * LDT + k + lk];
            b[t] = Bm[(qc + 16 * t + li) * LDT + k + lk];
        }
        for (int ti = 0; ti < 2; ++ti)
            for (int tj = 0; tj < 2; ++tj)
                acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
    }
}

// load rows [r0, r0+64) x columns [c0, c0+kk) of a column-major matrix into LDS row-major,
// zero outside [0, rmax) rows and beyond kk columns (up to 64)
__device__ inline void load_tile(double *S, const double *M, int64_t ld, int r0, int rmax, int c0, int kk) {
    // 16 loads per thread in flight before the LDS stores (256 threads x 16 = 64 x 64)
    double v[16];
    const int i = threadIdx.x % NB, k0 = threadIdx.x / NB;   // consecutive threads -> consecutive rows
    const int r = r0 + i;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int k = k0 + 4 * u;
        v[u] = (r < rmax && k < kk) ? M[r + ld * (c0 + k)] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) S[i * LDT + k0 + 4 * u] = v[u];
}

__global__ void __launch_bounds__(256)
k_potrf_diag(double *__restrict__ B, int64_t ldb, int j, int jb, double *__restrict__ Linv, int *__restrict__ fail) {
    __shared__ TileLds<64, 64> sh;
    const int tid = threadIdx.x;
    const int i0 = 4 * (tid / 16), j0 = 4 * (tid % 16);
    double a[4][4], r[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + u, k = j0 + v;
            a[u][v] = (i < jb && k <= i) ? B[(j + i) + ldb * (j + k)] : (i == k ? 1.0 : 0.0);
            r[u][v] = (i == k) ? 1.0 : 0.0;
        }
    int bad = 0;
    if (!chol_tile<4, 4, 16, true>(a, r, jb, sh, &bad)) {
        if (tid == 0) atomicCAS(fail, 0, j + bad + 1);
        return;
    }
    // the factor back into the lower part of the block, its inverse into Linv
    // (column-major 64 x 64, zero beyond the block)
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + u, k = j0 + v;
            if (i < jb && k <= i) B[(j + i) + ldb * (j + k)] = a[u][v];
            Linv[i + NB * k] = (i < jb && k < jb) ? r[u][v] : 0.0;
        }
}

__global__ void __launch_bounds__(256)
k_trsm_panel(double *__restrict__ B, int64_t ldb, int m, int j, int jb, const double *__restrict__ Linv) {
    // m here is the number of rows (the order of B, plus riding rows)
    __shared__ double A[NB * LDT];
    __shared__ double Bm[NB * LDT];
    const int r0 = j + jb + blockIdx.x * NB;
    load_tile(A, B, ldb, r0, m, j, jb);
    load_tile(Bm, Linv, NB, 0, NB, 0, NB);
    __syncthreads();
    d4 acc[2][2];
    tile_gemm_nt(A, Bm, jb, acc);
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    const int qr = 32 * (w % 2), qc = 32 * (w / 2);
    for (int ti = 0; ti < 2; ++ti)
        for (int tj = 0; tj < 2; ++tj)
            for (int r = 0; r < 4; ++r) {
                const int i = qr + 16 * ti + 4 * r + lane / 16;
                const int k = qc + 16 * tj + lane % 16;
                if (r0 + i < m && k < jb) B[(r0 + i) + ldb * (j + k)] = acc[ti][tj][r];
            }
}

__global__ void __launch_bounds__(256)
k_syrk_tiles(double *__restrict__ B, int64_t ldb, int rows, int m, int j, int jb) {
    __shared__ double A[NB * LDT];
    __shared__ double Bm[NB * LDT];
    const int ti = blockIdx.x, tk = blockIdx.y;
    if (tk > ti) return;
    const int base = j + jb;
    const int I0 = base + ti * NB, K0 = base + tk * NB;
    load_tile(A, B, ldb, I0, rows, j, jb);
    load_tile(Bm, B, ldb, K0, m, j, jb);
    __syncthreads();
    d4 acc[2][2];
    tile_gemm_nt(A, Bm, jb, acc);
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    const int qr = 32 * (w % 2), qc = 32 * (w / 2);
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c)
            for (int r = 0; r < 4; ++r) {
                const int gi = I0 + qr + 16 * a + 4 * r + lane / 16;
                const int gk = K0 + qc + 16 * c + lane % 16;
                if (gi < rows && gk < m && gi >= gk) B[gi + ldb * gk] -= acc[a][c][r];
            }
}

// backward step of R^T x = y over block J: x_J = Linv_J^T y_J, then
// y_c -= R(J, c)^T x_J for every column c before J (one wave per column)
__global__ void __launch_bounds__(256)
k_trsv_bwd_wave(const double *__restrict__ R, int64_t ldb, int j, int jb, const double *__restrict__ Linv,
                double *__restrict__ y, double *__restrict__ x) {
    __shared__ double xs[NB];
    const int tid = threadIdx.x;
    if (tid < jb) {
        double s = 0.0;
        for (int k = tid; k < jb; ++k) s += Linv[k + NB * tid] * y[j + k];
        xs[tid] = s;
    }
    __syncthreads();
    if (blockIdx.x == 0 && tid < jb) x[j + tid] = xs[tid];
    const int lane = tid % 64;
    const double xl = lane < jb ? xs[lane] : 0.0;
    for (int c = blockIdx.x * 4 + tid / 64; c < j; c += gridDim.x * 4) {
        double v = lane < jb ? R[(j + lane) + ldb * c] * xl : 0.0;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) y[c] -= v;
    }
}

// forward step: x_J = Linv_J y_J ; y_i -= R(i, J) x_J for i beyond J
__global__ void __launch_bounds__(256)
k_trsv_fwd(const double *__restrict__ R, int64_t ldb, int m, int j, int jb, const double *__restrict__ Linv,
           double *__restrict__ y, double *__restrict__ x) {
    __shared__ double xs[NB];
    const int tid = threadIdx.x;
    if (tid < jb) {
        double s = 0.0;
        for (int k = 0; k <= tid; ++k) s += Linv[tid + NB * k] * y[j + k];
        xs[tid] = s;
    }
    __syncthreads();
    if (blockIdx.x == 0 && tid < jb) x[j + tid] = xs[tid];
    for (int i = j + jb + blockIdx.x * blockDim.x + tid; i < m; i += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < jb; ++k) s += R[i + ldb * (j + k)] * xs[k];
        y[i] -= s;
    }
}

__global__ void k_copy(int m, const double *__restrict__ a, double *__restrict__ b) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) b[i] = a[i];
}

__global__ void k_scatter_strided(int m, const double *__restrict__ a, double *__restrict__ b, int64_t stride) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) b[i * stride] = a[i];
}

__global__ void k_copy_strided(int m, const double *__restrict__ a, int64_t stride, double *__restrict__ b) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) b[i] = a[i * stride];
}

}  // namespace

size_t potrf_work_doubles(int m) { return size_t((m + NB - 1) / NB) * NB * NB; }

void launch_potrf_rows(int m, int rows, double *B, int64_t ldb, double *work, int *fail, hipStream_t st) {
    for (int j = 0, s = 0; j < m; j += NB, ++s) {
        const int jb = (m - j < NB) ? (m - j) : NB;
        double *Linv = work + size_t(s) * NB * NB;
        hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, st, B, ldb, j, jb, Linv, fail);
        const int rest_rows = rows - j - jb;
        if (rest_rows <= 0) break;
        const int nt_r = (rest_rows + NB - 1) / NB;
        hipLaunchKernelGGL(k_trsm_panel, dim3(nt_r), dim3(256), 0, st, B, ldb, rows, j, jb, Linv);
        const int rest_cols = m - j - jb;
        if (rest_cols <= 0) continue;
        const int nt_c = (rest_cols + NB - 1) / NB;
        hipLaunchKernelGGL(k_syrk_tiles, dim3(nt_r, nt_c), dim3(256), 0, st, B, ldb, rows, m, j, jb);
    }
}

void launch_potrf(int m, double *B, int64_t ldb, double *work, int *fail, hipStream_t st) {
    launch_potrf_rows(m, m, B, ldb, work, fail, st);
}

void launch_potrs_bwd(int m, const double *R, int64_t ldb, const double *dinv, const double *u, int64_t ustride,
                      double *y, double *x, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_strided, dim3((m + 255) / 256), dim3(256), 0, st, m, u, ustride, y);
    const int nsteps = (m + NB - 1) / NB;
    for (int s = nsteps - 1; s >= 0; --s) {
        const int j = s * NB;
        const int jb = (m - j < NB) ? (m - j) : NB;
        int grid = (j + 3) / 4;
        if (grid < 1) grid = 1;
        if (grid > 1024) grid = 1024;
        hipLaunchKernelGGL(k_trsv_bwd_wave, dim3(grid), dim3(256), 0, st, R, ldb, j, jb,
                           dinv + size_t(s) * NB * NB, y, x);
    }
}

void launch_potrs(int m, const double *R, int64_t ldb, const double *dinv, const double *g, double *y, double *x,
                  hipStream_t st) {
    // forward: R u = g  (u into x), with y as the running right-hand side
    hipLaunchKernelGGL(k_copy, dim3((m + 255) / 256), dim3(256), 0, st, m, g, y);
    for (int j = 0, s = 0; j < m; j += NB, ++s) {
        const int jb = (m - j < NB) ? (m - j) : NB;
        const int rest = m - j - jb;
        const int grid = rest > 0 ? (rest + 255) / 256 : 1;
        hipLaunchKernelGGL(k_trsv_fwd, dim3(grid < 256 ? grid : 256), dim3(256), 0, st, R, ldb, m, j, jb,
                           dinv + size_t(s) * NB * NB, y, x);
    }
    launch_potrs_bwd(m, R, ldb, dinv, x, 1, y, x, st);
}

void launch_set_row(int m, const double *g, double *row, int64_t stride, hipStream_t st) {
    hipLaunchKernelGGL(k_scatter_strided, dim3((m + 255) / 256), dim3(256), 0, st, m, g, row, stride);
}

}  // namespace sdpc
