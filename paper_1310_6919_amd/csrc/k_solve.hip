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
// block step is two small dense products (k_inv_solve_mma, k_inv_solve), or
// one product with the block's G = [D^{-1}; P21 D^{-1}] (k_walk_g, blocks at
// most 32 wide and 64 high).  The next block's operands are loaded while the
// current block is processed, so a walk pays one memory latency at its start
// instead of one per block.  Finally the lower triangle is mirrored to make the
// output symmetric: by a separate pass after k_inv_solve_mma and k_inv_solve, while
// k_walk_g stores each entry below the diagonal at both places as it is found.
//
// The earlier factorisation X^ = L^T D L (Section 2.1, eq. sparse_fact) runs
// through the same walks with the sparse unit-lower L^{-1} as the factor: the
// forward walk gives L e_k, the block-diagonal D (w x w per storage block,
// zero between supernodes) multiplies each block's part of it before it is
// stored (in k_walk_g through the top block of the forward operand), and the
// backward walk applies L^T.
#include <algorithm>

#include "kernels.h"

namespace sdpc {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));   // one MFMA accumulator

constexpr int kThreads = 256;
constexpr int kPanelMax = 4096;                       // h * w doubles of one panel (enforced at analysis)
constexpr int kDinvMax = 32 * 32;                     // w * w doubles of one diagonal inverse
constexpr int kPanelPer = kPanelMax / kThreads;       // panel values per thread in flight
constexpr int kDinvPer = kDinvMax / kThreads;         // inverse values per thread in flight

struct BlockDesc {
    int F, w, h;
    int64_t r0;
    const double *P, *D;
};

__device__ inline BlockDesc block_desc(int b, const int *bl_first, const int64_t *bl_rptr, const int64_t *bl_off,
                                       const int64_t *bl_dinv, const double *L, const double *Dinv) {
    BlockDesc d;
    d.F = bl_first[b];
    d.w = bl_first[b + 1] - d.F;
    d.r0 = bl_rptr[b];
    d.h = int(bl_rptr[b + 1] - d.r0);
    d.P = L + bl_off[b];
    d.D = Dinv + bl_dinv[b];
    return d;
}

// Loads of a block's panel and inverse into registers (issued, not waited for).
__device__ inline void fetch_block(const BlockDesc &d, double (&rp)[kPanelPer], double (&rd)[kDinvPer]) {
    const int hw = d.h * d.w, ww = d.w * d.w;
#pragma unroll
    for (int u = 0; u < kPanelPer; ++u) {
        const int i = threadIdx.x + u * kThreads;
        rp[u] = i < hw ? d.P[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kDinvPer; ++u) {
        const int i = threadIdx.x + u * kThreads;
        rd[u] = i < ww ? d.D[i] : 0.0;
    }
}

// The same loads with clamped indices instead of guards: no branches, so the
// compiler's wait counting stays exact and the loads remain in flight across the
// block step instead of being waited for at its first use of any register.
__device__ inline void fetch_block_nb(const BlockDesc &d, double (&rp)[kPanelPer], double (&rd)[kDinvPer]) {
    const int hw = d.h * d.w, ww = d.w * d.w;
#pragma unroll
    for (int u = 0; u < kPanelPer; ++u) rp[u] = d.P[min(int(threadIdx.x) + u * kThreads, hw - 1)];
#pragma unroll
    for (int u = 0; u < kDinvPer; ++u) rd[u] = d.D[min(int(threadIdx.x) + u * kThreads, ww - 1)];
}

__device__ inline void put_block(const BlockDesc &d, const double (&rp)[kPanelPer], const double (&rd)[kDinvPer],
                                 double *Pn, double *Dn) {
    const int hw = d.h * d.w, ww = d.w * d.w;
#pragma unroll
    for (int u = 0; u < kPanelPer; ++u) {
        const int i = threadIdx.x + u * kThreads;
        if (i < hw) Pn[i] = rp[u];
    }
#pragma unroll
    for (int u = 0; u < kDinvPer; ++u) {
        const int i = threadIdx.x + u * kThreads;
        if (i < ww) Dn[i] = rd[u];
    }
}

template <int T>
__global__ void __launch_bounds__(kThreads)
k_inv_solve(int n, int nb, int maxw, int maxh, int pcap, const int *__restrict__ bl_first, const int64_t *__restrict__ bl_rptr,
            const int64_t *__restrict__ bl_off, const int *__restrict__ bl_subfirst,
            const int *__restrict__ bl_fslot, const int *__restrict__ bl_bslot,
            const int64_t *__restrict__ bl_dinv, const int *__restrict__ col_block, int nfwd, int nbwd,
            const double *__restrict__ L0, const double *__restrict__ Dinv0, double *__restrict__ out0,
            const double *__restrict__ L1, const double *__restrict__ Dinv1, double *__restrict__ out1,
            const double *__restrict__ Dm0, const double *__restrict__ Dm1) {
    // blockIdx.y picks one of two independent factors (they share the block layout),
    // so both inverses are formed by one launch and its workgroups interleave
    const double *L = blockIdx.y ? L1 : L0;
    const double *Dinv = blockIdx.y ? Dinv1 : Dinv0;
    double *out = blockIdx.y ? out1 : out0;
    const double *Dm = blockIdx.y ? Dm1 : Dm0;   // block diagonal between the walks, or null
    extern __shared__ double sm[];
    double *const Pbuf0 = sm, *const Pbuf1 = sm + pcap;      // pcap >= every h * w
    double *const Dbuf0 = sm + 2 * pcap, *const Dbuf1 = sm + 2 * pcap + maxw * maxw;
    double *accf = sm + 2 * pcap + 2 * maxw * maxw;          // nfwd * T
    double *accb = accf + nfwd * T;                          // nbwd * T
    double *v = accb + nbwd * T;                             // maxw * T
    double *xo = v + maxw * T;                               // maxw * T
    int *const slots0 = reinterpret_cast<int *>(xo + maxw * T), *const slots1 = slots0 + maxh;
    constexpr int RG = kThreads / T;
    const int tid = threadIdx.x;
    const int tc = tid % T;
    const int tr = tid / T;
    const int k0 = blockIdx.x * T;
    const int kend = min(n, k0 + T);
    for (int i = tid; i < (nfwd + nbwd) * T; i += kThreads) accf[i] = 0.0;
    const int b0 = col_block[k0];
    // a block takes part in the forward walk only if its elimination subtree meets the tile
    auto active = [&](int b) {
        const int F = bl_first[b], w = bl_first[b + 1] - F;
        return !(bl_subfirst[b] > kend - 1 || F + w - 1 < k0);
    };
    auto next_active = [&](int b) {
        for (++b; b < nb; ++b)
            if (active(b)) return b;
        return nb;
    };
    double rp[kPanelPer], rd[kDinvPer];
    // ------------------------------------------------------------ forward
    int cur = 0;
    int b = active(b0) ? b0 : next_active(b0);
    if (b < nb) {
        const BlockDesc d = block_desc(b, bl_first, bl_rptr, bl_off, bl_dinv, L, Dinv);
        fetch_block(d, rp, rd);
        put_block(d, rp, rd, Pbuf0, Dbuf0);
        for (int i = tid; i < d.h; i += kThreads) slots0[i] = bl_fslot[d.r0 + i];
    }
    __syncthreads();
    // Each dense product of a block step is computed in 2 x 2 register blocks
    // (two rows, two right-hand sides) so that every pair of operands read from LDS
    // feeds four multiply-adds.  The inverse D^{-1} of a diagonal block is stored
    // lower triangular with explicit zeros above the diagonal, so its products can
    // run over all w columns with a uniform bound.
    constexpr int TP = T / 2;
    while (b < nb) {
        const BlockDesc d = block_desc(b, bl_first, bl_rptr, bl_off, bl_dinv, L, Dinv);
        const int bn = next_active(b);
        BlockDesc dn{};
        if (bn < nb) {
            dn = block_desc(bn, bl_first, bl_rptr, bl_off, bl_dinv, L, Dinv);
            fetch_block(dn, rp, rd);   // in flight during this block's work
        }
        const double *Pn = ((cur) ? Pbuf1 : Pbuf0), *Dn = ((cur) ? Dbuf1 : Dbuf0);
        const int *fsl = ((cur) ? slots1 : slots0);
        const int F = d.F, w = d.w, h = d.h, hw = h - w;
        int fsn = -1;   // slot id of the next block's row tid, loaded with its panel
        if (bn < nb && tid < dn.h) fsn = bl_fslot[dn.r0 + tid];
        for (int i = tr; i < w; i += RG) {
            const int fs = fsl[i];
            double val = 0.0;
            if (fs >= 0) {
                val = accf[fs * T + tc];
                accf[fs * T + tc] = 0.0;
            }
            if (F + i == k0 + tc) val += 1.0;
            v[i * T + tc] = val;
        }
        __syncthreads();
        // xo = D^{-1} v (w x T), written to the output columns as well
        for (int blk = tid; blk < ((w + 1) / 2) * TP; blk += kThreads) {
            const int i0 = 2 * (blk / TP), c0 = 2 * (blk % TP), i1 = i0 + 1;
            const bool r1 = i1 < w;
            double s00 = 0.0, s01 = 0.0, s10 = 0.0, s11 = 0.0;
#pragma unroll 8
            for (int j = 0; j < w; ++j) {
                const double d0 = Dn[i0 + w * j], d1 = r1 ? Dn[i1 + w * j] : 0.0;
                const double v0 = v[j * T + c0], v1 = v[j * T + c0 + 1];
                s00 = fma(d0, v0, s00);
                s01 = fma(d0, v1, s01);
                s10 = fma(d1, v0, s10);
                s11 = fma(d1, v1, s11);
            }
            xo[i0 * T + c0] = s00;
            xo[i0 * T + c0 + 1] = s01;
            if (!Dm && k0 + c0 < n) out[int64_t(n) * (k0 + c0) + F + i0] = s00;
            if (!Dm && k0 + c0 + 1 < n) out[int64_t(n) * (k0 + c0 + 1) + F + i0] = s01;
            if (r1) {
                xo[i1 * T + c0] = s10;
                xo[i1 * T + c0 + 1] = s11;
                if (!Dm && k0 + c0 < n) out[int64_t(n) * (k0 + c0) + F + i1] = s10;
                if (!Dm && k0 + c0 + 1 < n) out[int64_t(n) * (k0 + c0 + 1) + F + i1] = s11;
            }
        }
        __syncthreads();
        if (Dm) {   // the forward result stored for the backward walk is D_b xo
            const double *Db = Dm + bl_dinv[b];
            for (int blk = tid; blk < ((w + 1) / 2) * TP; blk += kThreads) {
                const int i0 = 2 * (blk / TP), c0 = 2 * (blk % TP), i1 = i0 + 1;
                const bool r1 = i1 < w;
                double s00 = 0.0, s01 = 0.0, s10 = 0.0, s11 = 0.0;
                for (int j = 0; j < w; ++j) {
                    const double d0 = Db[i0 + w * j], d1 = r1 ? Db[i1 + w * j] : 0.0;
                    const double v0 = xo[j * T + c0], v1 = xo[j * T + c0 + 1];
                    s00 = fma(d0, v0, s00);
                    s01 = fma(d0, v1, s01);
                    s10 = fma(d1, v0, s10);
                    s11 = fma(d1, v1, s11);
                }
                if (k0 + c0 < n) out[int64_t(n) * (k0 + c0) + F + i0] = s00;
                if (k0 + c0 + 1 < n) out[int64_t(n) * (k0 + c0 + 1) + F + i0] = s01;
                if (r1) {
                    if (k0 + c0 < n) out[int64_t(n) * (k0 + c0) + F + i1] = s10;
                    if (k0 + c0 + 1 < n) out[int64_t(n) * (k0 + c0 + 1) + F + i1] = s11;
                }
            }
        }
        // pending updates of the rows below the block: acc(U) -= P21 xo
        for (int blk = tid; blk < ((hw + 1) / 2) * TP; blk += kThreads) {
            const int a0 = 2 * (blk / TP), c0 = 2 * (blk % TP), a1 = a0 + 1;
            const bool r1 = a1 < hw;
            double s00 = 0.0, s01 = 0.0, s10 = 0.0, s11 = 0.0;
#pragma unroll 8
            for (int j = 0; j < w; ++j) {
                const double p0 = Pn[(w + a0) + h * j], p1 = r1 ? Pn[(w + a1) + h * j] : 0.0;
                const double x0 = xo[j * T + c0], x1 = xo[j * T + c0 + 1];
                s00 = fma(p0, x0, s00);
                s01 = fma(p0, x1, s01);
                s10 = fma(p1, x0, s10);
                s11 = fma(p1, x1, s11);
            }
            const int f0 = fsl[w + a0];
            accf[f0 * T + c0] -= s00;
            accf[f0 * T + c0 + 1] -= s01;
            if (r1) {
                const int f1 = fsl[w + a1];
                accf[f1 * T + c0] -= s10;
                accf[f1 * T + c0 + 1] -= s11;
            }
        }
        if (bn < nb) {
            put_block(dn, rp, rd, ((cur ^ 1) ? Pbuf1 : Pbuf0), ((cur ^ 1) ? Dbuf1 : Dbuf0));
            if (tid < dn.h) ((cur ^ 1) ? slots1 : slots0)[tid] = fsn;
        }
        __syncthreads();
        cur ^= 1;
        b = bn;
    }
    // ------------------------------------------------------------ backward
    b = nb - 1;
    {
        const BlockDesc d = block_desc(b, bl_first, bl_rptr, bl_off, bl_dinv, L, Dinv);
        fetch_block(d, rp, rd);
        put_block(d, rp, rd, ((cur) ? Pbuf1 : Pbuf0), ((cur) ? Dbuf1 : Dbuf0));
        for (int i = tid; i < d.h; i += kThreads) ((cur) ? slots1 : slots0)[i] = bl_bslot[d.r0 + i];
    }
    __syncthreads();
    for (; b >= b0; --b) {
        const BlockDesc d = block_desc(b, bl_first, bl_rptr, bl_off, bl_dinv, L, Dinv);
        BlockDesc dn{};
        int bsn = -1;
        if (b > b0) {
            dn = block_desc(b - 1, bl_first, bl_rptr, bl_off, bl_dinv, L, Dinv);
            fetch_block(dn, rp, rd);
            if (tid < dn.h) bsn = bl_bslot[dn.r0 + tid];
        }
        const double *Pn = ((cur) ? Pbuf1 : Pbuf0), *Dn = ((cur) ? Dbuf1 : Dbuf0);
        const int *bsl = ((cur) ? slots1 : slots0);
        const int F = d.F, w = d.w, h = d.h, hw = h - w;
        const bool fwd_active = active(b);
        // v = z - P21^T acc(U), with z the forward result of the block (zero if inactive)
        for (int blk = tid; blk < ((w + 1) / 2) * TP; blk += kThreads) {
            const int j0 = 2 * (blk / TP), c0 = 2 * (blk % TP), j1 = j0 + 1;
            const bool r1 = j1 < w;
            const bool ok0 = fwd_active && k0 + c0 < n, ok1 = fwd_active && k0 + c0 + 1 < n;
            double s00 = ok0 ? out[int64_t(n) * (k0 + c0) + F + j0] : 0.0;
            double s01 = ok1 ? out[int64_t(n) * (k0 + c0 + 1) + F + j0] : 0.0;
            double s10 = (r1 && ok0) ? out[int64_t(n) * (k0 + c0) + F + j1] : 0.0;
            double s11 = (r1 && ok1) ? out[int64_t(n) * (k0 + c0 + 1) + F + j1] : 0.0;
#pragma unroll 8
            for (int a = 0; a < hw; ++a) {
                const double *q = accb + bsl[w + a] * T + c0;
                const double p0 = Pn[(w + a) + h * j0], p1 = r1 ? Pn[(w + a) + h * j1] : 0.0;
                const double q0 = q[0], q1 = q[1];
                s00 = fma(-p0, q0, s00);
                s01 = fma(-p0, q1, s01);
                s10 = fma(-p1, q0, s10);
                s11 = fma(-p1, q1, s11);
            }
            v[j0 * T + c0] = s00;
            v[j0 * T + c0 + 1] = s01;
            if (r1) {
                v[j1 * T + c0] = s10;
                v[j1 * T + c0 + 1] = s11;
            }
        }
        __syncthreads();
        // x = D^{-T} v (column i of D^{-1}, rows j >= i; zeros above the diagonal)
        for (int blk = tid; blk < ((w + 1) / 2) * TP; blk += kThreads) {
            const int i0 = 2 * (blk / TP), c0 = 2 * (blk % TP), i1 = i0 + 1;
            const bool r1 = i1 < w;
            double s00 = 0.0, s01 = 0.0, s10 = 0.0, s11 = 0.0;
#pragma unroll 8
            for (int j = 0; j < w; ++j) {
                const double d0 = Dn[j + w * i0], d1 = r1 ? Dn[j + w * i1] : 0.0;
                const double v0 = v[j * T + c0], v1 = v[j * T + c0 + 1];
                s00 = fma(d0, v0, s00);
                s01 = fma(d0, v1, s01);
                s10 = fma(d1, v0, s10);
                s11 = fma(d1, v1, s11);
            }
            const int bs0 = bsl[i0];
            if (k0 + c0 < n) out[int64_t(n) * (k0 + c0) + F + i0] = s00;
            if (k0 + c0 + 1 < n) out[int64_t(n) * (k0 + c0 + 1) + F + i0] = s01;
            if (bs0 >= 0) {
                accb[bs0 * T + c0] = s00;
                accb[bs0 * T + c0 + 1] = s01;
            }
            if (r1) {
                const int bs1 = bsl[i1];
                if (k0 + c0 < n) out[int64_t(n) * (k0 + c0) + F + i1] = s10;
                if (k0 + c0 + 1 < n) out[int64_t(n) * (k0 + c0 + 1) + F + i1] = s11;
                if (bs1 >= 0) {
                    accb[bs1 * T + c0] = s10;
                    accb[bs1 * T + c0 + 1] = s11;
                }
            }
        }
        if (b > b0) {
            put_block(dn, rp, rd, ((cur ^ 1) ? Pbuf1 : Pbuf0), ((cur ^ 1) ? Dbuf1 : Dbuf0));
            if (tid < dn.h) ((cur ^ 1) ? slots1 : slots0)[tid] = bsn;
        }
        __syncthreads();
        cur ^= 1;
    }
}

// Descriptor of a storage block, staged in LDS by the MFMA variant below so that
// a walk step costs no dependent memory round trip before its panel is fetched.
struct SolveDesc {
    int F, w, h, sub;
    int64_t r0, poff, doff;
};

constexpr int kRhs = 16;   // right-hand sides per workgroup on the MFMA variant

// One 16 x 16 tile of sum_k A(row, k) B(k, col) over at most 32 values of k on
// the FP64 MFMA.  fa(k) and fb(k) return this lane's operands for
// k = 4 ks + l / 16 (zero where k is out of range).  All operands are read
// first, then two accumulators take alternate k-steps, which halves the chain
// of dependent MFMAs.
template <typename FA, typename FB>
__device__ inline d4 mma32(FA fa, FB fb) {
    const int lq = (threadIdx.x & 63) >> 4;
    double xa[8], zb[8];
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
        xa[ks] = fa(4 * ks + lq);
        zb[ks] = fb(4 * ks + lq);
    }
    d4 a0 = d4{0.0, 0.0, 0.0, 0.0}, a1 = a0;
#pragma unroll
    for (int ks = 0; ks < 8; ks += 2) {
        a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[ks], zb[ks], a0, 0, 0, 0);
        a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[ks + 1], zb[ks + 1], a1, 0, 0, 0);
    }
    return a0 + a1;
}

// mma32 with this lane's B operands already in registers (zb[ks] for
// k = 4 ks + l / 16).
template <typename FA>
__device__ inline d4 mma32_breg(FA fa, const double (&zb)[8]) {
    const int lq = (threadIdx.x & 63) >> 4;
    double xa[8];
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) xa[ks] = fa(4 * ks + lq);
    d4 a0 = d4{0.0, 0.0, 0.0, 0.0}, a1 = a0;
#pragma unroll
    for (int ks = 0; ks < 8; ks += 2) {
        a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[ks], zb[ks], a0, 0, 0, 0);
        a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[ks + 1], zb[ks + 1], a1, 0, 0, 0);
    }
    return a0 + a1;
}

// The same walks with T = 16 right-hand sides, blocks of width <= 32, and every
// dense product of a block step on the FP64 MFMA (16 x 16 x 4; lane l supplies
// A(l % 16, l / 16) and B(l / 16, l % 16), element r of the result is
// C(4 r + l / 16, l % 16)).  Products whose result goes to the output columns are
// formed transposed (right-hand side as the row index), so the 16 lanes of a row
// group write 16 consecutive rows of one output column.
__global__ void __launch_bounds__(kThreads)
k_inv_solve_mma(int n, int nb, int maxw, int maxh, int pcap, const int *__restrict__ bl_first,
                const int64_t *__restrict__ bl_rptr, const int64_t *__restrict__ bl_off,
                const int *__restrict__ bl_subfirst, const int *__restrict__ bl_fslot,
                const int *__restrict__ bl_bslot, const int64_t *__restrict__ bl_dinv,
                const int *__restrict__ col_block, int nfwd, int nbwd, const double *__restrict__ L0,
                const double *__restrict__ Dinv0, double *__restrict__ out0, const double *__restrict__ L1,
                const double *__restrict__ Dinv1, double *__restrict__ out1, const double *__restrict__ Dm0,
                const double *__restrict__ Dm1) {
    constexpr int T = kRhs;
    const double *L = blockIdx.y ? L1 : L0;
    const double *Dinv = blockIdx.y ? Dinv1 : Dinv0;
    double *out = blockIdx.y ? out1 : out0;
    const double *Dm = blockIdx.y ? Dm1 : Dm0;   // block diagonal between the walks, or null
    extern __shared__ double sm[];
    double *const Pbuf0 = sm, *const Pbuf1 = sm + pcap;
    double *const Dbuf0 = sm + 2 * pcap, *const Dbuf1 = sm + 2 * pcap + maxw * maxw;
    double *accf = sm + 2 * pcap + 2 * maxw * maxw;   // nfwd * T
    double *accb = accf + nfwd * T;                   // nbwd * T
    double *v = accb + nbwd * T;                      // maxw * T
    double *xo = v + maxw * T;                        // maxw * T
    SolveDesc *desc = reinterpret_cast<SolveDesc *>(xo + maxw * T);
    int *const slots0 = reinterpret_cast<int *>(desc + nb), *const slots1 = slots0 + maxh;
    const int tid = threadIdx.x;
    const int wv = tid >> 6, l = tid & 63, li = l & 15, lq = l >> 4;
    const int tc = tid % T, tr = tid / T;
    constexpr int RG = kThreads / T;
    const int k0 = blockIdx.x * T;
    const int kend = min(n, k0 + T);
    for (int i = tid; i < (nfwd + nbwd) * T; i += kThreads) accf[i] = 0.0;
    for (int b = tid; b < nb; b += kThreads) {
        SolveDesc e;
        e.F = bl_first[b];
        e.w = bl_first[b + 1] - e.F;
        e.r0 = bl_rptr[b];
        e.h = int(bl_rptr[b + 1] - e.r0);
        e.sub = bl_subfirst[b];
        e.poff = bl_off[b];
        e.doff = bl_dinv[b];
        desc[b] = e;
    }
    __syncthreads();
    const int b0 = col_block[k0];
    auto active = [&](int b) {
        const SolveDesc &e = desc[b];
        return !(e.sub > kend - 1 || e.F + e.w - 1 < k0);
    };
    auto next_active = [&](int b) {
        for (++b; b < nb; ++b)
            if (active(b)) return b;
        return nb;
    };
    auto bdesc = [&](int b) {
        const SolveDesc &e = desc[b];
        BlockDesc d;
        d.F = e.F;
        d.w = e.w;
        d.h = e.h;
        d.r0 = e.r0;
        d.P = L + e.poff;
        d.D = Dinv + e.doff;
        return d;
    };
    double rp[kPanelPer], rd[kDinvPer];
    // with D: this lane's operands of D_b (waves 0 and 1), D(16 wv + l % 16, 4 ks + l / 16),
    // for the current block and, prefetched with its panel, the next one
    double dmr[8], dmn[8];
    auto fetch_dm = [&](int bb, double (&z)[8]) {
        const SolveDesc &e = desc[bb];
        const int i = min(16 * wv + li, e.w - 1);
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) z[ks] = Dm[e.doff + i + e.w * min(4 * ks + lq, e.w - 1)];
    };
    // ------------------------------------------------------------ forward
    int cur = 0;
    int b = active(b0) ? b0 : next_active(b0);
    if (b < nb) {
        const BlockDesc d = bdesc(b);
        fetch_block(d, rp, rd);
        put_block(d, rp, rd, Pbuf0, Dbuf0);
        for (int i = tid; i < d.h; i += kThreads) slots0[i] = bl_fslot[d.r0 + i];
        if (Dm && wv < 2) fetch_dm(b, dmr);
    }
    __syncthreads();
    while (b < nb) {
        const BlockDesc d = bdesc(b);
        const int bn = next_active(b);
        BlockDesc dn{};
        int fsn = -1;
        if (bn < nb) {
            dn = bdesc(bn);
            fetch_block_nb(dn, rp, rd);   // in flight during this block's work
            fsn = bl_fslot[dn.r0 + min(tid, dn.h - 1)];
            if (Dm && wv < 2) fetch_dm(bn, dmn);
        }
        const double *Pn = ((cur) ? Pbuf1 : Pbuf0), *Dn = ((cur) ? Dbuf1 : Dbuf0);
        const int *fsl = ((cur) ? slots1 : slots0);
        const int F = d.F, w = d.w, h = d.h, hw = h - w;
        const int w1 = w - 1, hw1 = max(hw - 1, 0);   // clamps: operand reads stay in range
#pragma unroll
        for (int u = 0; u < 32 / RG; ++u) {   // w <= 32
            const int i = tr + RG * u;
            if (i < w) {
                const int fs = fsl[i];
                double val = 0.0;
                if (fs >= 0) {
                    val = accf[fs * T + tc];
                    accf[fs * T + tc] = 0.0;
                }
                if (F + i == k0 + tc) val += 1.0;
                v[i * T + tc] = val;
            }
        }
        __syncthreads();
        // xo = D^{-1} v, as xo^T = v^T D^{-T}: element (c, i)
        if (wv < (w + 15) / 16) {
            const int i = 16 * wv + li, ic = min(i, w1);
            const d4 acc = mma32(
                [&](int k) {
                    const double x = v[min(k, w1) * T + li];
                    return (k < w) ? x : 0.0;
                },
                [&](int k) {
                    const double z = Dn[ic + w * min(k, w1)];
                    return (k < w && i < w) ? z : 0.0;
                });
            if (i < w) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = 4 * r + lq;
                    xo[i * T + c] = acc[r];
                    if (!Dm && k0 + c < n) out[int64_t(n) * (k0 + c) + F + i] = acc[r];
                }
            }
        }
        __syncthreads();
        // with D: the forward result stored for the backward walk is D_b xo, as
        // (D_b xo)^T = xo^T D_b^T: element (c, i)
        if (Dm && wv < (w + 15) / 16) {
            const int i = 16 * wv + li;
            double zb[8];
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) zb[ks] = (4 * ks + lq < w && i < w) ? dmr[ks] : 0.0;
            const d4 acc = mma32_breg(
                [&](int k) {
                    const double x = xo[min(k, w1) * T + li];
                    return (k < w) ? x : 0.0;
                },
                zb);
            if (i < w) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = 4 * r + lq;
                    if (k0 + c < n) out[int64_t(n) * (k0 + c) + F + i] = acc[r];
                }
            }
        }
        // pending updates of the rows below the block: acc(U) -= P21 xo, element (a, c)
        for (int rt = wv; rt < (hw + 15) / 16; rt += 4) {
            const int a = 16 * rt + li, ac = min(a, hw1);
            const d4 acc = mma32(
                [&](int k) {
                    const double x = Pn[(w + ac) + h * min(k, w1)];
                    return (a < hw && k < w) ? x : 0.0;
                },
                [&](int k) {
                    const double z = xo[min(k, w1) * T + li];
                    return (k < w) ? z : 0.0;
                });
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ar = 16 * rt + 4 * r + lq;
                if (ar < hw) accf[fsl[w + ar] * T + li] -= acc[r];
            }
        }
        if (bn < nb) {
            put_block(dn, rp, rd, ((cur ^ 1) ? Pbuf1 : Pbuf0), ((cur ^ 1) ? Dbuf1 : Dbuf0));
            if (tid < dn.h) ((cur ^ 1) ? slots1 : slots0)[tid] = fsn;
            if (Dm) {
#pragma unroll
                for (int ks = 0; ks < 8; ++ks) dmr[ks] = dmn[ks];
            }
        }
        __syncthreads();
        cur ^= 1;
        b = bn;
    }
    // ------------------------------------------------------------ backward
    b = nb - 1;
    {
        const BlockDesc d = bdesc(b);
        fetch_block(d, rp, rd);
        put_block(d, rp, rd, ((cur) ? Pbuf1 : Pbuf0), ((cur) ? Dbuf1 : Dbuf0));
        for (int i = tid; i < d.h; i += kThreads) ((cur) ? slots1 : slots0)[i] = bl_bslot[d.r0 + i];
    }
    // forward result z of a block in the layout of the transposed products:
    // element r of lane (wv, l) is z(16 wv + li, 4 r + lq); zero if the block was
    // not on the forward walk
    auto load_z = [&](int bb, double (&z)[4]) {
        const SolveDesc &e = desc[bb];
        const bool on = active(bb);
        const int j = 16 * wv + li;
        const int jc = min(j, e.w - 1);   // clamped: every load is in bounds, selects afterwards
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = 4 * r + lq;
            const double zz = out[int64_t(n) * min(k0 + c, n - 1) + e.F + jc];
            z[r] = (on && wv < 2 && j < e.w && k0 + c < n) ? zz : 0.0;
        }
    };
    double zc[4], zn[4];
    load_z(b, zc);
    __syncthreads();
    for (; b >= b0; --b) {
        const BlockDesc d = bdesc(b);
        BlockDesc dn{};
        int bsn = -1;
        if (b > b0) {
            dn = bdesc(b - 1);
            fetch_block_nb(dn, rp, rd);
            bsn = bl_bslot[dn.r0 + min(tid, dn.h - 1)];
            load_z(b - 1, zn);
        }
        const double *Pn = ((cur) ? Pbuf1 : Pbuf0), *Dn = ((cur) ? Dbuf1 : Dbuf0);
        const int *bsl = ((cur) ? slots1 : slots0);
        const int F = d.F, w = d.w, h = d.h, hw = h - w;
        // v = z - P21^T acc(U), as v^T = z^T - acc(U)^T P21: element (c, j)
        if (wv < (w + 15) / 16) {
            const int j = 16 * wv + li, jc = min(j, w - 1), hw1 = max(hw - 1, 0);
            d4 acc = d4{0.0, 0.0, 0.0, 0.0};
            for (int a0 = 0; a0 < hw; a0 += 32)
                acc += mma32(
                    [&](int k) {
                        const int a = a0 + k;
                        const double x = accb[bsl[w + min(a, hw1)] * T + li];
                        return (a < hw) ? x : 0.0;
                    },
                    [&](int k) {
                        const int a = a0 + k;
                        const double z = Pn[(w + min(a, hw1)) + h * jc];
                        return (a < hw && j < w) ? z : 0.0;
                    });
            if (j < w) {
#pragma unroll
                for (int r = 0; r < 4; ++r) v[j * T + 4 * r + lq] = zc[r] - acc[r];
            }
        }
        __syncthreads();
        // x = D^{-T} v, as x^T = v^T D^{-1}: element (c, i)
        if (wv < (w + 15) / 16) {
            const int i = 16 * wv + li, ic = min(i, w - 1);
            const d4 acc = mma32(
                [&](int j) {
                    const double x = v[min(j, w - 1) * T + li];
                    return (j < w) ? x : 0.0;
                },
                [&](int j) {
                    const double z = Dn[min(j, w - 1) + w * ic];
                    return (j < w && i < w) ? z : 0.0;
                });
            if (i < w) {
                const int bs = bsl[i];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = 4 * r + lq;
                    if (k0 + c < n) out[int64_t(n) * (k0 + c) + F + i] = acc[r];
                    if (bs >= 0) accb[bs * T + c] = acc[r];
                }
            }
        }
        if (b > b0) {
            put_block(dn, rp, rd, ((cur ^ 1) ? Pbuf1 : Pbuf0), ((cur ^ 1) ? Dbuf1 : Dbuf0));
            if (tid < dn.h) ((cur ^ 1) ? slots1 : slots0)[tid] = bsn;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) zc[r] = zn[r];
        __syncthreads();
        cur ^= 1;
    }
}

// ---------------------------------------------------------------------------
// The same walks with one product per block step.  Per storage block
//   G_b = [ D_b^{-1} ; P21_b D_b^{-1} ]     (h x w, the panel's layout; k_dinv)
// holds both halves of a forward step: G_b v_b gives z_b = D_b^{-1} v_b in its first
// w rows (the forward result) and P21_b z_b in the others (the updates of the rows
// below).  The backward step is x_b = D_b^{-T} (z_b - P21_b^T x_below) =
// G_b^T [z_b; -x_below].  Each block step is therefore one MFMA product (16 x 16
// output tiles, one per wave forward, two waves backward), reading its right-hand
// side from the LDS slots and writing its results back, then one barrier.  The
// next block's operands (G, slot ids, the forward result read by the backward step)
// are loaded into registers in the MFMA layout while the current step runs, so
// nothing but the pending rows is staged in LDS.
// Pending forward updates are not zeroed when consumed: every slot records the
// last block that wrote it, and its value counts only if that block is not older
// than the first block that updates the slot's current row (blocks a tile skips
// write nothing).  The host frees a slot one block after its last use (SolveSlots),
// so no step reads a slot as one of its own rows while writing it as a row below.
// The output is stored symmetric: an entry (i, j) below the diagonal at (i, j) and
// (j, i), entries above it not at all (the forward results z, parked in `out` for
// the backward walk, vanish there and are taken as zeros).
// Limits: every block at most 32 columns wide and 64 rows high.
struct WalkDesc {
    int F, w, h, sub;
};

constexpr int kWalkWmax = 32, kWalkHmax = 64;
typedef int i4 __attribute__((ext_vector_type(4)));

// two workgroups per compute unit (at most 256 registers per lane): at n = 12000 the
// 1500 tiles of both factors need the second slot
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2)))
k_walk_g(int n, int nb, const int *__restrict__ bl_first, const int64_t *__restrict__ bl_rptr,
         const int *__restrict__ bl_subfirst, const int *__restrict__ wk_fs, const int *__restrict__ wk_fb,
         const int *__restrict__ wk_bs, const int *__restrict__ col_block, int nfwd, int nbwd,
         const double *__restrict__ G0, double *__restrict__ out0, const double *__restrict__ G1,
         double *__restrict__ out1) {
    constexpr int T = kRhs;
    const double *G = blockIdx.y ? G1 : G0;
    double *out = blockIdx.y ? out1 : out0;
    // at least one slot of each kind, so that the clamped slot 0 of a lane without a
    // slot is always a valid address
    const int nf1 = max(nfwd, 1), nb1 = max(nbwd, 1);
    extern __shared__ double sm[];
    double *accf = sm;                                   // nf1 x T pending forward updates
    double *accb = accf + size_t(nf1) * T;               // nb1 x T finished backward rows
    WalkDesc *desc = reinterpret_cast<WalkDesc *>(accb + size_t(nb1) * T);
    int *lwb = reinterpret_cast<int *>(desc + nb);       // nf1: last block that wrote each slot
    const int tid = threadIdx.x;
    const int wv = tid >> 6, l = tid & 63, li = l & 15, lq = l >> 4;
    const int k0 = blockIdx.x * T;
    const int kend = min(n, k0 + T);
    for (int i = tid; i < nf1; i += kThreads) lwb[i] = -1;
    for (int b = tid; b < nb; b += kThreads) {
        WalkDesc e;
        e.F = bl_first[b];
        e.w = bl_first[b + 1] - e.F;
        e.h = int(bl_rptr[b + 1] - bl_rptr[b]);
        e.sub = bl_subfirst[b];
        desc[b] = e;
    }
    __syncthreads();
    auto active = [&](int b) {
        const WalkDesc &e = desc[b];
        return !(e.sub > kend - 1 || e.F + e.w - 1 < k0);
    };
    auto next_active = [&](int b) {
        for (++b; b < nb; ++b)
            if (active(b)) return b;
        return nb;
    };
    // ------------------------------------------------------------ forward
    // lane operands of a forward step, wave wv owning output rows 16 wv .. 16 wv + 15,
    // each a few contiguous vector loads from the lane-ordered G and row lists (zero
    // and -1 outside the block): g[ks] = G(16 wv + li, 4 ks + lq); vs / vb: slot and
    // first updating block of row 4 ks + lq; os / ob: the same for row 16 wv + 4 r + lq
    struct Fwd {
        double g[8];
        int vs[8], vb[8], os[4], ob[4];
    };
    auto fetch_fwd = [&](int bb, Fwd &f) {
        const double2 *gp = reinterpret_cast<const double2 *>(G + size_t(bb) * 4096 + size_t(wv * 64 + l) * 8);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double2 t = gp[u];
            f.g[2 * u] = t.x;
            f.g[2 * u + 1] = t.y;
        }
        const i4 *fsp = reinterpret_cast<const i4 *>(wk_fs + size_t(bb) * 64 + lq * 16);
        const i4 *fbp = reinterpret_cast<const i4 *>(wk_fb + size_t(bb) * 64 + lq * 16);
        const i4 s0 = fsp[0], s1 = fsp[1], so = fsp[wv], b0v = fbp[0], b1v = fbp[1], bo = fbp[wv];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            f.vs[u] = s0[u];
            f.vs[4 + u] = s1[u];
            f.vb[u] = b0v[u];
            f.vb[4 + u] = b1v[u];
            f.os[u] = so[u];
            f.ob[u] = bo[u];
        }
    };
    const int b0 = col_block[k0];
    int b = active(b0) ? b0 : next_active(b0);
    int b1 = b < nb ? next_active(b) : nb;
    // operands two blocks ahead: a ring of three register sets, the loads of a block in
    // flight for two steps
    Fwd fa, fb, fc;
    if (b < nb) fetch_fwd(b, fa);
    if (b1 < nb) fetch_fwd(b1, fb);
    auto fstep = [&](const Fwd &cur, Fwd &pre) {
        const int F = desc[b].F, w = desc[b].w, h = desc[b].h;
        const int b2 = b1 < nb ? next_active(b1) : nb;
        fetch_fwd(b2 < nb ? b2 : b, pre);   // in flight during this step and the next
        // v: the pending updates of the block's own rows plus e_k
        double v[8];
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            const int k = 4 * ks + lq;
            const int sv = (k < w) ? cur.vs[ks] : -1;
            const int sc = max(sv, 0);
            const double x = accf[sc * T + li];
            const bool have = sv >= 0 && lwb[sc] >= cur.vb[ks];
            v[ks] = (have ? x : 0.0) + ((k < w && F + k == k0 + li) ? 1.0 : 0.0);
        }
        if (16 * wv < h) {   // uniform
            // two independent chains; k-steps beyond the block's columns add nothing
            d4 a[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) a[t] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < 8; ++ks)
                if (4 * ks < w) a[ks & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur.g[ks], v[ks], a[ks & 1], 0, 0, 0);
            const d4 acc = a[0] + a[1];
            // element r: row 16 wv + 4 r + lq of G v, right-hand side li; every lane of a
            // row reads the row's slot stamp before any of them rewrites it
            int os[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int orow = 16 * wv + 4 * r + lq;
                os[r] = (orow >= w) ? cur.os[r] : -1;   // -1 beyond the block already
                const int sc = max(os[r], 0);
                const double old = (os[r] >= 0 && lwb[sc] >= cur.ob[r]) ? accf[sc * T + li] : 0.0;
                if (orow < w) {   // z, lower triangle only (z vanishes above the diagonal)
                    if (k0 + li < n && F + orow >= k0 + li) out[int64_t(n) * (k0 + li) + F + orow] = acc[r];
                } else if (os[r] >= 0) {
                    accf[sc * T + li] = old - acc[r];
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (os[r] >= 0) lwb[os[r]] = b;
        }
        __syncthreads();
        b = b1;
        b1 = b2;
    };
    for (;;) {
        if (b >= nb) break;
        fstep(fa, fc);
        if (b >= nb) break;
        fstep(fb, fa);
        if (b >= nb) break;
        fstep(fc, fb);
    }
    // the forward results in `out`, stored by other threads, are read below
    __syncthreads();
    // ------------------------------------------------------------ backward
    // Waves 0, 1 compute (output rows 16 wv .. 16 wv + 15) from lane-ordered operands:
    // ga[ks] = G(4 ks + lq, 16 wv + li); us[ks]: backward slot of row 4 ks + lq; os[r]:
    // backward slot of output row 16 wv + 4 r + lq.
    // Waves 2, 3 load the forward results z of the blocks to come: the columns of
    // `out` lie n doubles apart and were written long before, so these loads miss in
    // L2.  Block q's z is loaded at the step of block q + 3 (register set q & 1),
    // written into the LDS ring slot q & 1 at the step of block q + 1, and read at
    // the step of block q; zero where the block was not on the forward walk.
    struct Bwd {
        double ga[16];
        int us[16], os[4];
    };
    auto fetch_bwd = [&](int bb, Bwd &f) {
        const double2 *gp =
            reinterpret_cast<const double2 *>(G + size_t(bb) * 4096 + 2048 + size_t(wv * 64 + l) * 16);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double2 t = gp[u];
            f.ga[2 * u] = t.x;
            f.ga[2 * u + 1] = t.y;
        }
        const i4 *bsp = reinterpret_cast<const i4 *>(wk_bs + size_t(bb) * 64 + lq * 16);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const i4 t = bsp[u];
#pragma unroll
            for (int j = 0; j < 4; ++j) f.us[4 * u + j] = t[j];
        }
        const i4 to = bsp[wv];
#pragma unroll
        for (int j = 0; j < 4; ++j) f.os[j] = to[j];
    };
    constexpr int ZLD = 33;   // ring slot: z(k, c) at c * ZLD + k, 16 x 32
    double *zr = reinterpret_cast<double *>(lwb + nf1 + (nf1 & 1));
    const int lt = tid - 128;   // loader thread (waves 2, 3): entries lt + 128 j, row k = e % 32, column c = e / 32
    auto zload = [&](int q, double (&zs)[4]) {
        const WalkDesc e = desc[q];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int ent = lt + 128 * j, k = ent & 31, c = ent >> 5;
            zs[j] = out[int64_t(n) * min(k0 + c, n - 1) + e.F + min(k, e.w - 1)];
        }
    };
    auto zwrite = [&](int q, const double (&zs)[4]) {
        const WalkDesc e = desc[q];
        const bool on = active(q);
        double *zslot = zr + (q & 1) * (16 * ZLD);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int ent = lt + 128 * j, k = ent & 31, c = ent >> 5;
            zslot[c * ZLD + k] = (on && k < e.w && k0 + c < n && e.F + k >= k0 + c) ? zs[j] : 0.0;
        }
    };
    double zs0[4], zs1[4];   // loader register sets: block q in set q & 1
    b = nb - 1;
    // operands two blocks ahead, as in the forward walk
    Bwd xa, xb, xc;
    if (wv < 2) {
        fetch_bwd(b, xa);
        if (b - 1 >= b0) fetch_bwd(b - 1, xb);
    } else {
        if (b & 1) zload(b, zs1); else zload(b, zs0);
        if (b - 1 >= b0) {
            if ((b - 1) & 1) zload(b - 1, zs1); else zload(b - 1, zs0);
        }
        if (b & 1) zwrite(b, zs1); else zwrite(b, zs0);
        if (b - 2 >= b0) {
            if (b & 1) zload(b - 2, zs1); else zload(b - 2, zs0);
        }
    }
    __syncthreads();
    auto bstep = [&](const Bwd &bc, Bwd &pre) {
        const int F = desc[b].F, w = desc[b].w, h = desc[b].h;
        if (wv < 2) {
            fetch_bwd(b - 2 >= b0 ? b - 2 : b, pre);   // in flight during this step and the next
            if (16 * wv < w) {   // uniform
                const double *zslot = zr + (b & 1) * (16 * ZLD);
                // two independent chains; k-steps beyond the block's rows add nothing
                d4 a[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) a[t] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < 16; ++kk) {
                    if (4 * kk < h) {   // uniform
                        const int k = 4 * kk + lq;
                        const int sv = (k >= w) ? bc.us[kk] : -1;   // -1 beyond the block already
                        const double x = accb[max(sv, 0) * T + li];
                        const double zz = (kk < 8) ? zslot[li * ZLD + (kk < 8 ? k : 0)] : 0.0;
                        const double u = (k < w) ? zz : (sv >= 0 ? -x : 0.0);
                        a[kk & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(bc.ga[kk], u, a[kk & 1], 0, 0, 0);
                    }
                }
                const d4 acc = a[0] + a[1];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int orow = 16 * wv + 4 * r + lq;
                    if (orow < w) {
                        // (i, j) below the diagonal is stored twice, at (i, j) and (j, i)
                        // (rows of the output: 16 consecutive columns per lane group);
                        // above it nothing: the column of i stores it
                        const int i = F + orow, j = k0 + li;
                        if (j < n && i >= j) out[int64_t(n) * j + i] = acc[r];
                        if (j < n && i > j) out[j + int64_t(n) * i] = acc[r];
                        if (bc.os[r] >= 0) accb[bc.os[r] * T + li] = acc[r];
                    }
                }
            }
        } else if (b - 1 >= b0) {
            // write block b - 1's z (set (b - 1) & 1), then load block b - 3 into that set
            if ((b - 1) & 1) {
                zwrite(b - 1, zs1);
                if (b - 3 >= b0) zload(b - 3, zs1);
            } else {
                zwrite(b - 1, zs0);
                if (b - 3 >= b0) zload(b - 3, zs0);
            }
        }
        __syncthreads();
        --b;
    };
    for (;;) {
        if (b < b0) break;
        bstep(xa, xc);
        if (b < b0) break;
        bstep(xb, xa);
        if (b < b0) break;
        bstep(xc, xb);
    }
}

// out(j, i) = out(i, j) for i > j, 32 x 32 tiles of the lower triangle
__global__ void __launch_bounds__(256) k_mirror(int n, double *__restrict__ out0, double *__restrict__ out1) {
    __shared__ double t[32][33];
    double *out = blockIdx.z ? out1 : out0;
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

int solve_pcap(const DevStruct &d) { return int(d.max_panel < 1 ? 1 : d.max_panel); }

size_t solve_lds(const DevStruct &d, int T) {
    return sizeof(double) * (size_t(2) * solve_pcap(d) + size_t(2) * d.max_w * d.max_w +
                             size_t(d.nfwd + d.nbwd) * T + size_t(2) * d.max_w * T) +
           sizeof(int) * 2 * size_t(d.max_h);   // slot ids of the rows of the two buffered blocks
}

size_t solve_lds_mma(const DevStruct &d) {
    return solve_lds(d, kRhs) + sizeof(SolveDesc) * size_t(d.nb);
}

size_t walk_g_lds(const DevStruct &d) {
    const size_t nf1 = size_t(std::max(d.wk_nfwd, 1)), nb1 = size_t(std::max(d.wk_nbwd, 1));
    return sizeof(double) * (nf1 + nb1) * kRhs + sizeof(WalkDesc) * size_t(d.nb) + sizeof(int) * (nf1 + (nf1 & 1)) +
           sizeof(double) * 2 * 16 * 33;   // the ring of forward results read by the backward walk
}

bool solve_mma_ok(const DevStruct &d) {
    return d.max_panel <= kPanelMax && d.max_w <= 32 && d.max_h <= kThreads && solve_lds_mma(d) <= 64 * 1024;
}

}  // namespace

bool walk_g_ok(const DevStruct &d) {
    return d.max_w <= kWalkWmax && d.max_h <= kWalkHmax && d.wk_fs != nullptr && walk_g_lds(d) <= 64 * 1024;
}

int solve_tile_width(const DevStruct &d) {
    if (d.max_panel > kPanelMax || d.max_w * d.max_w > kDinvMax || d.max_h > kThreads) return 0;
    for (int T : {16, 8, 4, 2})   // products run on pairs of right-hand sides
        if (solve_lds(d, T) <= 64 * 1024) return T;
    return 0;
}

void launch_inverse_by_solves(const DevStruct &d, const double *L0, const double *Dinv0, double *out0,
                              const double *L1, const double *Dinv1, double *out1, hipStream_t st,
                              const double *Dm0, const double *Dm1, const double *G0, const double *G1) {
    const int nf = L1 ? 2 : 1;
    const int nt = (d.n + 31) / 32;
    if (!d.solve_generic && G0 && (nf == 1 || G1) && walk_g_ok(d)) {   // any Dm is inside G
        hipLaunchKernelGGL(k_walk_g, dim3((d.n + kRhs - 1) / kRhs, nf), dim3(kThreads), walk_g_lds(d), st, d.n, d.nb,
                           d.bl_first, d.bl_rptr, d.bl_subfirst, d.wk_fs, d.wk_fb, d.wk_bs, d.col_block,
                           d.wk_nfwd, d.wk_nbwd, G0, out0, G1, out1);   // both triangles
        return;
    }
    if (!d.solve_generic && solve_mma_ok(d)) {
        hipLaunchKernelGGL(k_inv_solve_mma, dim3((d.n + kRhs - 1) / kRhs, nf), dim3(kThreads), solve_lds_mma(d), st,
                           d.n, d.nb, d.max_w, d.max_h, solve_pcap(d), d.bl_first, d.bl_rptr, d.bl_off,
                           d.bl_subfirst, d.bl_fslot, d.bl_bslot, d.bl_dinv, d.col_block, d.nfwd, d.nbwd, L0, Dinv0,
                           out0, L1, Dinv1, out1, Dm0, Dm1);
        hipLaunchKernelGGL(k_mirror, dim3(nt, nt, nf), dim3(256), 0, st, d.n, out0, out1);
        return;
    }
    const int T = solve_tile_width(d);
    const int grid = (d.n + T - 1) / T;
    const size_t lds = solve_lds(d, T);
#define SDPC_SOLVE(TT)                                                                                     \
    hipLaunchKernelGGL(k_inv_solve<TT>, dim3(grid, nf), dim3(kThreads), lds, st, d.n, d.nb, d.max_w, d.max_h, \
                       solve_pcap(d), d.bl_first, d.bl_rptr, d.bl_off, d.bl_subfirst, d.bl_fslot, d.bl_bslot,   \
                       d.bl_dinv, d.col_block, d.nfwd, d.nbwd, L0, Dinv0, out0, L1, Dinv1, out1, Dm0, Dm1)
    switch (T) {
        case 16: SDPC_SOLVE(16); break;
        case 8: SDPC_SOLVE(8); break;
        case 4: SDPC_SOLVE(4); break;
        default: SDPC_SOLVE(2); break;
    }
#undef SDPC_SOLVE
    hipLaunchKernelGGL(k_mirror, dim3(nt, nt, nf), dim3(256), 0, st, d.n, out0, out1);
}

}  // namespace sdpc
