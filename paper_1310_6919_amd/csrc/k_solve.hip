// Multi-right-hand-side sparse substitutions (types (iv) and (v) of
// Section 3.1): out(:, k) = L^{-T} L^{-1} e_k for every k, i.e. the columns
// Lhat^{-T} Lhat^{-1} e_k = X^ e_k and N^{-T} N^{-1} e_k = Y^{-1} e_k that
// eq. newSCM2 and eq. newdX2 consume.  On the GPU every column is computed
// once per iteration and kept in HBM (the paper recomputes them per SCM
// column because a CPU cannot hold the dense X^).
//
// One workgroup owns a tile of T consecutive right-hand sides [k0, k0+T):
//   forward   walk the storage blocks from block(k0) upwards; a block is
//             visited only if its elimination subtree meets the tile (the
//             others see a zero right-hand side); pending updates of rows
//             that are not yet final live in LDS slots (assigned on the host
//             so that rows alive at the same time never share a slot);
//   backward  walk the blocks from the root down to block(k0): only rows
//             >= k0 (and the rest of block(k0)) are needed, and the backward
//             substitution restricted to those rows is self-contained; values
//             still read by lower blocks stay in LDS slots.
// The diagonal blocks are applied through their explicit inverses, so each
// block step is two small dense products.  Panels are staged through LDS.
// Finally the lower triangle is mirrored to make the output symmetric.
#include "kernels.h"

namespace sdpc {

namespace {

constexpr int kThreads = 256;
constexpr int kPanelMax = 4096;   // h * w doubles of one staged panel

template <int T>
__global__ void __launch_bounds__(kThreads)
k_inv_solve(int n, int nb, int maxw, const int *__restrict__ bl_first, const int64_t *__restrict__ bl_rptr,
            const int64_t *__restrict__ bl_off, const int *__restrict__ bl_subfirst,
            const int *__restrict__ bl_fslot, const int *__restrict__ bl_bslot,
            const int64_t *__restrict__ bl_dinv, const int *__restrict__ col_block, int nfwd, int nbwd,
            const double *__restrict__ L, const double *__restrict__ Dinv, double *__restrict__ out) {
    extern __shared__ double sm[];
    double *Pn = sm;                                  // kPanelMax
    double *Dn = Pn + kPanelMax;                      // maxw * maxw
    double *accf = Dn + maxw * maxw;                  // nfwd * T
    double *accb = accf + nfwd * T;                   // nbwd * T
    double *v = accb + nbwd * T;                      // maxw * T
    double *xo = v + maxw * T;                        // maxw * T
    constexpr int RG = kThreads / T;
    const int tid = threadIdx.x;
    const int tc = tid % T;
    const int tr = tid / T;
    const int k0 = blockIdx.x * T;
    const int kend = min(n, k0 + T);
    const bool colok = (k0 + tc) < n;
    double *outc = out + int64_t(n) * (k0 + tc);
    for (int i = tid; i < (nfwd + nbwd) * T; i += kThreads) accf[i] = 0.0;
    const int b0 = col_block[k0];
    __syncthreads();
    // ------------------------------------------------------------ forward
    for (int b = b0; b < nb; ++b) {
        const int F = bl_first[b];
        const int w = bl_first[b + 1] - F;
        if (bl_subfirst[b] > kend - 1 || F + w - 1 < k0) continue;   // subtree misses the tile
        const int64_t r0 = bl_rptr[b];
        const int h = int(bl_rptr[b + 1] - r0);
        const double *P = L + bl_off[b];
        const double *D = Dinv + bl_dinv[b];
        stage_lds<8>(Pn, P, h * w);
        stage_lds<4>(Dn, D, w * w);
        for (int i = tr; i < w; i += RG) {
            const int fs = bl_fslot[r0 + i];
            double val = 0.0;
            if (fs >= 0) {
                val = accf[fs * T + tc];
                accf[fs * T + tc] = 0.0;
            }
            if (F + i == k0 + tc) val += 1.0;
            v[i * T + tc] = val;
        }
        __syncthreads();
        for (int i = tr; i < w; i += RG) {
            double s = 0.0;
            for (int j = 0; j <= i; ++j) s += Dn[i + w * j] * v[j * T + tc];
            xo[i * T + tc] = s;
            if (colok) outc[F + i] = s;
        }
        __syncthreads();
        for (int a = tr; a < h - w; a += RG) {
            double s = 0.0;
            for (int j = 0; j < w; ++j) s += Pn[(w + a) + h * j] * xo[j * T + tc];
            const int fs = bl_fslot[r0 + w + a];
            accf[fs * T + tc] -= s;
        }
        __syncthreads();
    }
    // ------------------------------------------------------------ backward
    for (int b = nb - 1; b >= b0; --b) {
        const int F = bl_first[b];
        const int w = bl_first[b + 1] - F;
        const bool fwd_active = !(bl_subfirst[b] > kend - 1 || F + w - 1 < k0);
        const int64_t r0 = bl_rptr[b];
        const int h = int(bl_rptr[b + 1] - r0);
        const double *P = L + bl_off[b];
        const double *D = Dinv + bl_dinv[b];
        stage_lds<8>(Pn, P, h * w);
        stage_lds<4>(Dn, D, w * w);
        __syncthreads();
        for (int j = tr; j < w; j += RG) {
            double s = (fwd_active && colok) ? outc[F + j] : 0.0;
            for (int a = 0; a < h - w; ++a) {
                const int bs = bl_bslot[r0 + w + a];
                s -= Pn[(w + a) + h * j] * accb[bs * T + tc];
            }
            v[j * T + tc] = s;
        }
        __syncthreads();
        for (int i = tr; i < w; i += RG) {
            double s = 0.0;
            for (int j = i; j < w; ++j) s += Dn[j + w * i] * v[j * T + tc];
            if (colok) outc[F + i] = s;
            const int bs = bl_bslot[r0 + i];
            if (bs >= 0) accb[bs * T + tc] = s;
        }
        __syncthreads();
    }
}

// out(j, i) = out(i, j) for i > j, 32 x 32 tiles of the lower triangle
__global__ void __launch_bounds__(256) k_mirror(int n, double *__restrict__ out) {
    __shared__ double t[32][33];
    const int bi = blockIdx.x, bj = blockIdx.y;   // tile row, tile column
    if (bi < bj) return;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    for (int r = ty; r < 32; r += 8) {
        const int i = bi * 32 + r, j = bj * 32 + tx;
        t[r][tx] = (i < n && j < n) ? out[i + int64_t(n) * j] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = bi * 32 + tx;    // source row
        const int j = bj * 32 + r;     // source column
        if (i < n && j < n && i > j) out[j + int64_t(n) * i] = t[tx][r];
    }
}

size_t solve_lds(const DevStruct &d, int T) {
    return sizeof(double) * (size_t(kPanelMax) + size_t(d.max_w) * d.max_w +
                             size_t(d.nfwd + d.nbwd) * T + size_t(2) * d.max_w * T);
}

}  // namespace

int solve_tile_width(const DevStruct &d) {
    if (int64_t(d.max_h) * d.max_w > kPanelMax) return 0;
    for (int T : {16, 8, 4, 2, 1})
        if (solve_lds(d, T) <= 64 * 1024) return T;
    return 0;
}

void launch_inverse_by_solves(const DevStruct &d, const double *L, const double *Dinv, double *out,
                              hipStream_t st) {
    const int T = solve_tile_width(d);
    const int grid = (d.n + T - 1) / T;
    const size_t lds = solve_lds(d, T);
#define SDPC_SOLVE(TT)                                                                                   \
    hipLaunchKernelGGL(k_inv_solve<TT>, dim3(grid), dim3(kThreads), lds, st, d.n, d.nb, d.max_w,         \
                       d.bl_first, d.bl_rptr, d.bl_off, d.bl_subfirst, d.bl_fslot, d.bl_bslot, d.bl_dinv, \
                       d.col_block, d.nfwd, d.nbwd, L, Dinv, out)
    switch (T) {
        case 16: SDPC_SOLVE(16); break;
        case 8: SDPC_SOLVE(8); break;
        case 4: SDPC_SOLVE(4); break;
        case 2: SDPC_SOLVE(2); break;
        default: SDPC_SOLVE(1); break;
    }
#undef SDPC_SOLVE
    const int nt = (d.n + 31) / 32;
    hipLaunchKernelGGL(k_mirror, dim3(nt, nt), dim3(256), 0, st, d.n, out);
}

}  // namespace sdpc
