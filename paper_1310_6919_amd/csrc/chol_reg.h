// Register-resident Cholesky of a small symmetric matrix (order c <= 64) by one
// 256-thread workgroup, shared by the dense SCM diagonal blocks, Algorithm 1
// and the clique-wise step-length test.
//
// Thread (i, q) = (tid / 4, tid % 4) holds row i at columns q, q + 4, ..., q + 60
// in a[0..15] (entries above the diagonal are zero).  Only the scaled pivot
// column (colc), the finished row of L^{-1} (rowc) and the next pivot (piv)
// pass through LDS.  Every LDS value a step needs is read before any update, and
// the updates are masked multiply-adds, so the LDS latency is paid once per step
// instead of once per element.
#pragma once
#include <hip/hip_runtime.h>

namespace sdpc {

// 1/sqrt(d) from the hardware estimate refined by two Newton steps
// (y <- y (3 - d y^2) / 2), and sqrt(d) = d / sqrt(d); a short dependent chain
// compared with a correctly rounded square root followed by a division.
__device__ inline void rsqrt_pivot(double d, double &rd, double &inv) {
    double y = __builtin_amdgcn_rsq(d);
    y = y * fma(-0.5 * d, y * y, 1.5);
    y = y * fma(-0.5 * d, y * y, 1.5);
    inv = y;
    rd = d * y;
}

struct CholLds {
    double colc[64];
    double rowc[64];
    double piv[2];
};

// Factorises in place: on success a[] holds L (A = L L^T) and, when INV, r[]
// holds L^{-1} (r must start as the identity rows).  Returns false (uniformly
// across the workgroup) when a pivot is not positive; *bad_pivot gets its index.
template <bool INV>
__device__ inline bool chol_reg(double a[16], double r[16], int c, CholLds &sh, int *bad_pivot) {
    const int tid = threadIdx.x, i = tid >> 2, q = tid & 3;
    if (tid == 0) sh.piv[0] = a[0];
    __syncthreads();
    for (int k = 0; k < c; ++k) {
        const double d = sh.piv[k & 1];
        if (!(d > 0.0) || !isfinite(d)) {
            *bad_pivot = k;
            return false;   // uniform: every thread read the same pivot
        }
        double rd, inv;
        rsqrt_pivot(d, rd, inv);
        // column k: owners scale their entry below the pivot and publish it
        if (q == (k & 3)) {
            const int tk = k >> 2;
#pragma unroll
            for (int t = 0; t < 16; ++t)
                if (t == tk) {
                    if (i > k && i < c) {
                        a[t] *= inv;
                        sh.colc[i] = a[t];
                    } else if (i == k) {
                        a[t] = rd;
                    }
                }
        }
        if (INV && i == k) {
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const double v = r[t] * inv;   // row k of L^{-1} is final
                r[t] = (q + 4 * t <= k) ? v : r[t];
                if (q + 4 * t <= k) sh.rowc[q + 4 * t] = v;
            }
        }
        __syncthreads();
        if (i > k && i < c) {
            const double l = sh.colc[i];
            double cv[16], rv[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                cv[t] = sh.colc[q + 4 * t];
                if (INV) rv[t] = sh.rowc[q + 4 * t];
            }
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int kk = q + 4 * t;
                const double la = (kk > k && kk <= i) ? l : 0.0;
                a[t] = fma(-la, cv[t], a[t]);
                if (INV) {
                    const double lr = (kk <= k) ? l : 0.0;
                    r[t] = fma(-lr, rv[t], r[t]);
                }
            }
        }
        if (i == k + 1 && q == ((k + 1) & 3)) {
            const int tk = (k + 1) >> 2;
#pragma unroll
            for (int t = 0; t < 16; ++t)
                if (t == tk) sh.piv[(k + 1) & 1] = a[t];
        }
        __syncthreads();
    }
    return true;
}

}  // namespace sdpc
