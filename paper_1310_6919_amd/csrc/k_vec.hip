// Assembly of matrices on the storage layout, state metrics, vector updates.
//
//   Y = A_0 - sum_k z_k A_k                      (dual slack, Section 1 (D))
//   G = A_0 - sum_k z_k A_k - Y                   (dual residual)
//   dY = G - sum_k dz_k A_k                       (Section 2.2, HKM direction)
// are all one gather per storage slot over the A_k entries that land there
// (fixed order, no atomics).
#include "kernels.h"

namespace sdpc {

namespace {

constexpr int kThreads = 256;

// out = a + b (b may be null: out = a)
__global__ void k_add(int64_t len, const double *__restrict__ a, const double *__restrict__ b,
                      double *__restrict__ out) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < len; i += int64_t(gridDim.x) * blockDim.x)
        out[i] = b ? a[i] + b[i] : a[i];
}

__global__ void k_assemble(int64_t nslot, const int64_t *__restrict__ ptr, const int *__restrict__ kk,
                           const double *__restrict__ val, const double *__restrict__ y, double a0,
                           double c1, const double *__restrict__ in1, double *__restrict__ out) {
    for (int64_t s = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; s < nslot;
         s += int64_t(gridDim.x) * blockDim.x) {
        double acc = 0.0;
        for (int64_t t = ptr[s]; t < ptr[s + 1]; ++t) {
            const int k = kk[t];
            const double coef = (k == 0) ? a0 : -y[k - 1];
            acc += coef * val[t];
        }
        if (in1) acc += c1 * in1[s];
        out[s] = acc;
    }
}

// Block-wide reductions (sum and max), blockDim = 1024.
__device__ double block_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (t < o) sh[t] += sh[t + o];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ double block_max(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (t < o) sh[t] = fmax(sh[t], sh[t + o]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// scal[0] = A_0 . X, scal[1] = b . z, scal[2] = max_k |b_k - A_k . X|,
// scal[3] = max |G|, scal[4] = X . Y (on E), scal[5] = 1 if anything non-finite.
// kMetricsGroups workgroups write partial results part[8 g + i]; k_metrics_final
// combines them in a fixed order.
constexpr int kMetricsGroups = 64;

// resid[k] = b_k - A_k . X for k < m: one wave per constraint, the entries split over
// the lanes and summed in a fixed order (a constraint can hold many entries)
__global__ void __launch_bounds__(256) k_con_resid(int m, const int64_t *__restrict__ con_ptr,
                                                 const int *__restrict__ con_slot, const double *__restrict__ con_val,
                                                 const double *__restrict__ b, const double *__restrict__ X,
                                                 double *__restrict__ resid) {
    const int lane = threadIdx.x & 63;
    const int waves = gridDim.x * (blockDim.x >> 6);
    for (int k = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); k < m; k += waves) {
        double a = 0.0;
        for (int64_t e = con_ptr[k + 1] + lane; e < con_ptr[k + 2]; e += 64) a = fma(con_val[e], X[con_slot[e]], a);
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
        if (lane == 0) resid[k] = b[k] - a;
    }
}

// Long constraints, chunk by chunk: workgroup c sums con_val[e] v(e) over the entries
// of chunk c, each thread over its entries in order, the threads combined in a fixed
// order (v(e) = v[con_slot[e]], or v(pi, pj) of a dense n x n matrix with DENSE)
template <bool DENSE>
__global__ void __launch_bounds__(256) k_con_chunk(const int *__restrict__ ch_con, const int64_t *__restrict__ ch_beg,
                                                 const int64_t *__restrict__ con_ptr, const int *__restrict__ con_slot,
                                                 const int *__restrict__ con_pi, const int *__restrict__ con_pj,
                                                 const double *__restrict__ con_val, const double *__restrict__ v,
                                                 int n, double *__restrict__ part) {
    __shared__ double ws[4];
    const int c = blockIdx.x, k = ch_con[c];
    const int64_t beg = ch_beg[c];
    const int64_t lim = beg + int64_t(kConChunk), end = (con_ptr[k + 2] < lim) ? con_ptr[k + 2] : lim;
    double a = 0.0;
    for (int64_t e = beg + threadIdx.x; e < end; e += 256) {
        const double x = DENSE ? v[con_pi[e] + int64_t(n) * con_pj[e]] : v[con_slot[e]];
        a = fma(con_val[e], x, a);
    }
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) part[c] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// out[k] = b_k - coef (the chunk sums of constraint k, in order) + add[k]
__global__ void __launch_bounds__(256) k_con_finish(int m, const int *__restrict__ ch_ptr,
                                                  const double *__restrict__ part, const double *__restrict__ b,
                                                  double coef, const double *__restrict__ add,
                                                  double *__restrict__ out) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < m; k += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int c = ch_ptr[k]; c < ch_ptr[k + 1]; ++c) s += part[c];
        out[k] = b[k] - coef * s + (add ? add[k] : 0.0);
    }
}

__global__ void __launch_bounds__(1024) k_metrics(int m, int64_t nslot, const int64_t *__restrict__ con_ptr,
                                                  const int *__restrict__ con_slot,
                                                  const double *__restrict__ con_val,
                                                  const double *__restrict__ b, const double *__restrict__ wE,
                                                  const double *__restrict__ X, const double *__restrict__ Y,
                                                  const double *__restrict__ z, const double *__restrict__ G,
                                                  const double *__restrict__ resid, double *__restrict__ part) {
    __shared__ double sh[1024];
    const int t = threadIdx.x;
    const int64_t i0 = int64_t(blockIdx.x) * blockDim.x + t, step = int64_t(gridDim.x) * blockDim.x;
    double pobj = 0.0, bz = 0.0, rmax = 0.0, gmax = 0.0, xy = 0.0;
    bool bad = false;
    // A_0 . X over all threads (A_0 carries the whole aggregate pattern)
    for (int64_t e = con_ptr[0] + i0; e < con_ptr[1]; e += step) pobj += con_val[e] * X[con_slot[e]];
    for (int64_t k = 1 + i0; k <= m; k += step) {
        rmax = fmax(rmax, fabs(resid[k - 1]));
        bz += b[k - 1] * z[k - 1];
        bad |= !isfinite(z[k - 1]);
    }
    for (int64_t s = i0; s < nslot; s += step) {
        const double w = wE[s];
        xy += w * X[s] * Y[s];
        gmax = fmax(gmax, fabs(G[s]));
        bad |= !(isfinite(X[s]) && isfinite(Y[s]));
    }
    pobj = block_sum(pobj, sh);
    bz = block_sum(bz, sh);
    rmax = block_max(rmax, sh);
    gmax = block_max(gmax, sh);
    xy = block_sum(xy, sh);
    const double nb = block_max(bad ? 1.0 : 0.0, sh);
    if (t == 0) {
        double *pp = part + 8 * blockIdx.x;
        pp[0] = pobj;
        pp[1] = bz;
        pp[2] = rmax;
        pp[3] = gmax;
        pp[4] = xy;
        pp[5] = nb;
    }
}

// ng <= kMetricsGroups; the partial results are staged in LDS by all lanes (one
// round of loads), then combined by one thread in group order
__global__ void __launch_bounds__(64) k_metrics_final(int ng, const double *__restrict__ part,
                                                      double *__restrict__ scal) {
    __shared__ double sp[8 * kMetricsGroups];
    for (int i = threadIdx.x; i < 8 * ng; i += blockDim.x) sp[i] = part[i];
    __syncthreads();
    if (threadIdx.x != 0) return;
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int g = 0; g < ng; ++g) {
        const double *pp = sp + 8 * g;
        v[0] += pp[0];
        v[1] += pp[1];
        v[2] = fmax(v[2], pp[2]);
        v[3] = fmax(v[3], pp[3]);
        v[4] += pp[4];
        v[5] = fmax(v[5], pp[5]);
    }
    for (int i = 0; i < 6; ++i) scal[i] = v[i];
}

// Step 4 with the step lengths still on the device: out = x + scale * alpha[0] * dx,
// unless the iteration has failed, i.e. one of the nflag failure flags is set or
// one of the two step lengths (alpha[0] and, when given, alpha2[0]) is not
// positive; then out = x (in place: untouched), so a failed step leaves the
// iterate as it was.
__global__ void k_axpy_checked(int64_t len, const double *x, const double *__restrict__ dx,
                               const double *__restrict__ alpha, const double *__restrict__ alpha2, double scale,
                               const int *__restrict__ flags, int nflag, double *out) {
    bool ok = alpha[0] > 0.0 && (!alpha2 || alpha2[0] > 0.0);
    for (int i = 0; i < nflag; ++i) ok = ok && flags[i] == 0;
    const double coef = scale * alpha[0];
    for (int64_t s = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; s < len;
         s += int64_t(gridDim.x) * blockDim.x) {
        if (ok)
            out[s] = fma(coef, dx[s], x[s]);   // the same rounding as the dual-step candidates
        else if (out != x)
            out[s] = x[s];
    }
}

// out = candidate sel[0] of a pool of ncand vectors of length len, where the
// index was left on the device as a double by an earlier kernel; a negative or
// out-of-range index leaves out as it is.
__global__ void k_copy_selected(int64_t len, const double *__restrict__ pool, const double *__restrict__ sel,
                                int ncand, double *__restrict__ out) {
    const double c = sel[0];
    if (!(c >= 0.0) || !(c < double(ncand))) return;
    const double *__restrict__ src = pool + int64_t(c) * len;
    for (int64_t s = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; s < len;
         s += int64_t(gridDim.x) * blockDim.x)
        out[s] = src[s];
}

// out(i, j) = in(pos[i], pos[j]): a dense n x n column-major matrix from the
// elimination order back to the original indices
__global__ void __launch_bounds__(256) k_unpermute(int n, const int *__restrict__ pos, const double *__restrict__ in,
                                                   double *__restrict__ out) {
    const int j = blockIdx.x;
    const int64_t pj = int64_t(pos[j]) * n;
    for (int i = blockIdx.y * blockDim.x + threadIdx.x; i < n; i += gridDim.y * blockDim.x)
        out[i + int64_t(n) * j] = in[pos[i] + pj];
}

__global__ void k_init(int64_t nslot, const double *__restrict__ wE, double lambda, double *X, double *Y,
                       int m, double *z) {
    // diagonal slots are exactly those with weight 1
    for (int64_t s = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; s < nslot;
         s += int64_t(gridDim.x) * blockDim.x) {
        const double v = (wE[s] == 1.0) ? lambda : 0.0;
        X[s] = v;
        Y[s] = v;
    }
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < m; k += int64_t(gridDim.x) * blockDim.x)
        z[k] = 0.0;
}

__global__ void k_mask(int64_t nslot, const double *__restrict__ wE, double *v) {
    for (int64_t s = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; s < nslot;
         s += int64_t(gridDim.x) * blockDim.x)
        if (wE[s] == 0.0) v[s] = 0.0;
}

int grid_for(int64_t len) {
    int64_t g = (len + kThreads - 1) / kThreads;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return int(g);
}

}  // namespace

void launch_assemble(const DevStruct &d, const double *y, double a0, double c1, const double *in1,
                     double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_assemble, dim3(grid_for(d.nslot)), dim3(kThreads), 0, st, d.nslot, d.asm_ptr,
                       d.asm_k, d.asm_val, y, a0, c1, in1, out);
}

size_t metrics_work_doubles(const DevStruct &d) {
    return size_t(8) * kMetricsGroups + size_t(d.m > 0 ? d.m : 1) + size_t(d.con_chunks);
}

bool launch_con_chunks(const DevStruct &d, bool dense, const double *v, double coef, const double *add,
                       double *out, double *work, hipStream_t st) {
    if (d.con_chunks <= 0 || d.m <= 0) return false;
    double *part = work + 8 * kMetricsGroups + d.m;
    if (dense)
        hipLaunchKernelGGL(k_con_chunk<true>, dim3(d.con_chunks), dim3(256), 0, st, d.ch_con, d.ch_beg, d.con_ptr,
                           d.con_slot, d.con_pi, d.con_pj, d.con_val, v, d.n, part);
    else
        hipLaunchKernelGGL(k_con_chunk<false>, dim3(d.con_chunks), dim3(256), 0, st, d.ch_con, d.ch_beg, d.con_ptr,
                           d.con_slot, d.con_pi, d.con_pj, d.con_val, v, d.n, part);
    hipLaunchKernelGGL(k_con_finish, dim3((d.m + 255) / 256), dim3(256), 0, st, d.m, d.ch_ptr, (const double *)part,
                       d.b, coef, add, out);
    return true;
}

void launch_metrics(const DevStruct &d, const double *X, const double *Y, const double *z, double *G,
                    double *scal, double *work, hipStream_t st) {
    // G = A_0 - sum z_k A_k - Y
    launch_assemble(d, z, 1.0, -1.0, Y, G, st);
    double *resid = work + 8 * kMetricsGroups;
    if (d.m > 0 && !launch_con_chunks(d, false, X, 1.0, nullptr, resid, work, st))
        hipLaunchKernelGGL(k_con_resid, dim3((d.m + 3) / 4 < 4096 ? (d.m + 3) / 4 : 4096), dim3(256), 0, st, d.m,
                           d.con_ptr, d.con_slot, d.con_val, d.b, X, resid);
    hipLaunchKernelGGL(k_metrics, dim3(kMetricsGroups), dim3(1024), 0, st, d.m, d.nslot, d.con_ptr, d.con_slot,
                       d.con_val, d.b, d.wE, X, Y, z, G, (const double *)resid, work);
    hipLaunchKernelGGL(k_metrics_final, dim3(1), dim3(64), 0, st, kMetricsGroups, (const double *)work, scal);
}

void launch_axpy_checked(int64_t len, const double *x, const double *dx, const double *alpha, const double *alpha2,
                         double scale, const int *flags, int nflag, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_axpy_checked, dim3(grid_for(len)), dim3(kThreads), 0, st, len, x, dx, alpha, alpha2, scale,
                       flags, nflag, out);
}

void launch_copy_selected(int64_t len, const double *pool, const double *sel, int ncand, double *out,
                          hipStream_t st) {
    if (len > 0)
        hipLaunchKernelGGL(k_copy_selected, dim3(grid_for(len)), dim3(kThreads), 0, st, len, pool, sel, ncand, out);
}

void launch_add(int64_t len, const double *a, const double *b, double *out, hipStream_t st) {
    if (len > 0)
        hipLaunchKernelGGL(k_add, dim3(grid_for(len)), dim3(kThreads), 0, st, len, a, b, out);
}

void launch_unpermute(const DevStruct &d, const double *in, double *out, hipStream_t st) {
    if (d.n <= 0) return;
    hipLaunchKernelGGL(k_unpermute, dim3(d.n, (d.n + 255) / 256), dim3(256), 0, st, d.n, d.pos, in, out);
}

void launch_init_point(const DevStruct &d, double lambda, double *X, double *Y, double *z, hipStream_t st) {
    hipLaunchKernelGGL(k_init, dim3(grid_for(d.nslot > d.m ? d.nslot : d.m)), dim3(kThreads), 0, st,
                       d.nslot, d.wE, lambda, X, Y, d.m, z);
}

void launch_mask_E(const DevStruct &d, double *v, hipStream_t st) {
    hipLaunchKernelGGL(k_mask, dim3(grid_for(d.nslot)), dim3(kThreads), 0, st, d.nslot, d.wE, v);
}

}  // namespace sdpc
