// Factorisations on the clique / block structure.
//
//  k_sn_chol      Y = N N^T, supernodal right-looking Cholesky on the storage
//                 blocks (type (v) of Section 3.1).  One workgroup walks the
//                 blocks in elimination order; each panel is factorised in LDS
//                 and its update is scattered into the ancestor panels through
//                 precomputed slots.  blockIdx.x selects a candidate
//                 Y + alpha_c dY, which turns the same kernel into a parallel
//                 positive-definiteness test for the dual step length
//                 (Section 2.2, Step 3).
//  k_sn_chol_wave the same for panels of at most 64 rows, one wave per
//                 candidate: rows in registers, the ancestors' update on the
//                 FP64 MFMA.
//  k_dinv         inverses of the diagonal blocks of a factor (used by the
//                 multi-right-hand-side substitutions) and, for the
//                 single-product walks, each block's G = [D^{-1}; P21 D^{-1}].
//  k_algorithm1   Algorithm 1: per clique C_r, the lower Cholesky factor of
//                 (Xbar(C_r, C_r))^{-1} without forming the inverse: the block
//                 in reversed order P_r Xbar P_r^T = M_r M_r^T gives it as
//                 P_r M_r^{-T} P_r^T, whose first |S_r| columns are
//                 Lhat(C_r, S_r).
//  k_alpha_cl     eq. primal_length2: per clique the largest alpha in (0, 1]
//                 keeping Xbar(C_r,C_r) + alpha dX(C_r,C_r) positive definite,
//                 found by bisection on the Cholesky test.
#include "chol_reg.h"
#include "kernels.h"

namespace sdpc {

namespace {

constexpr int kCholThreads = 256;

// Candidate step lengths of the dual positive-definiteness test.  Candidates
// c < ntest are the test points: round 0 is a logarithmic grid 1e-8 .. 1, later
// rounds an even grid inside the bracket (lo, hi) left by the previous round.
// Candidates c >= ntest are twins gamma * t of test points t: in round 0 one
// twin of t = 1, in later rounds one twin per test point.  The twin of the step
// finally taken is the factor of the next iterate Y + gamma alpha dY.
__device__ inline double cand_alpha(int c, int ntest, int round, double gamma, const double *bracket) {
    const bool twin = c >= ntest;
    const int t = twin ? (round == 0 ? ntest - 1 : c - ntest) : c;
    const double a = (round == 0) ? pow(10.0, -8.0 * double(ntest - 1 - t) / double(ntest - 1))
                                  : bracket[0] + (bracket[1] - bracket[0]) * double(t + 1) / double(ntest + 1);
    return twin ? gamma * a : a;
}

__global__ void __launch_bounds__(kCholThreads)
k_sn_chol(int nb, int64_t nslot, const double *__restrict__ wE, const int *__restrict__ bl_first, const int64_t *__restrict__ bl_rptr,
          const int64_t *__restrict__ bl_off, const int64_t *__restrict__ up_ptr,
          const int *__restrict__ up_pair, const int *__restrict__ up_slot, const double *__restrict__ Y,
          const double *__restrict__ dY, const double *__restrict__ bracket, int round, int ntest, double gamma,
          double *__restrict__ Lbase, int64_t stride, int *__restrict__ fail) {
    extern __shared__ double P[];
    __shared__ TileLds<64, 32> tsh;   // pivot columns of a panel with at most 64 rows
    __shared__ double colw[32];  // scaled pivot column (block width <= 32), tall panels
    const int tid = threadIdx.x;
    const int cand = blockIdx.x;
    double *L = Lbase + cand * stride;
    double al = 0.0;
    if (dY) {
        // the candidate's step length (bracket[2] != 0: settled, nothing to test)
        if (round > 0 && bracket[2] != 0.0) {
            if (tid == 0) fail[cand] = 0;
            return;
        }
        al = cand_alpha(cand, ntest, round, gamma, bracket);
    }
    // padding slots of the inputs are ignored (the factor stores an exact zero there)
    for (int64_t s = tid; s < nslot; s += blockDim.x)
        L[s] = (wE[s] == 0.0) ? 0.0 : (dY ? fma(al, dY[s], Y[s]) : Y[s]);
    __threadfence_block();
    __syncthreads();
    for (int b = 0; b < nb; ++b) {
        const int F = bl_first[b];
        const int w = bl_first[b + 1] - F;
        const int h = int(bl_rptr[b + 1] - bl_rptr[b]);
        const int64_t off = bl_off[b];
        stage_lds<16>(P, L + off, h * w);
        __syncthreads();
        // right-looking factorisation of the panel
        if (h <= 64) {
            // panel in registers: thread tiles of 2 rows x 4 columns over 64 x 32,
            // zeros outside the panel; the factor goes back into P
            const int i0 = 2 * (tid / 8), j0 = 4 * (tid % 8);
            double a[2][4], unused[2][4];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = i0 + u, k = j0 + v;
                    a[u][v] = (i < h && k < w && (i >= w || k <= i)) ? P[i + h * k] : 0.0;
                    unused[u][v] = 0.0;
                }
            int bad = 0;
            if (!chol_tile<2, 4, 8, false>(a, unused, w, tsh, &bad)) {
                if (tid == 0) fail[cand] = b + 1;
                return;   // uniform
            }
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = i0 + u, k = j0 + v;
                    if (i < h && k < w && (i >= w || k <= i)) P[i + h * k] = a[u][v];
                }
            __syncthreads();
        } else {
            // tall panels: entries stay in LDS; thread (row lane r, quarter q) updates
            // rows r, r + 64, ... at columns j + 1 + q, j + 5 + q, ...
            const int rl = tid & 63, q = tid >> 6;
            for (int j = 0; j < w; ++j) {
                const double d = P[j + h * j];
                if (!(d > 0.0) || !isfinite(d)) {
                    if (tid == 0) fail[cand] = b + 1;
                    return;
                }
                const double rd = sqrt(d);
                const double inv = 1.0 / rd;
                for (int k = j + 1 + tid; k < w; k += blockDim.x) colw[k] = P[k + h * j] * inv;
                for (int i = j + 1 + tid; i < h; i += blockDim.x) P[i + h * j] *= inv;
                __syncthreads();
                if (tid == 0) P[j + h * j] = rd;
                for (int i = j + 1 + rl; i < h; i += 64) {
                    const double lij = P[i + h * j];
                    const int kend = i < w ? i : w - 1;
                    double v[8];
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        const int k = j + 1 + q + 4 * t;
                        v[t] = (k <= kend) ? P[i + h * k] : 0.0;
                    }
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        const int k = j + 1 + q + 4 * t;
                        if (k <= kend) P[i + h * k] = v[t] - lij * colw[k];
                    }
                }
                __syncthreads();
            }
        }
        for (int i = tid; i < h * w; i += blockDim.x) L[off + i] = P[i];
        for (int64_t t = up_ptr[b] + tid; t < up_ptr[b + 1]; t += blockDim.x) {
            const int s = up_slot[t];
            if (s < 0) continue;
            const int pr = up_pair[t];
            const int ra = w + (pr & 0xffff), rc = w + (pr >> 16);
            double v = 0.0;
            for (int j = 0; j < w; ++j) v += P[ra + h * j] * P[rc + h * j];
            L[s] -= v;
        }
        __threadfence_block();
        __syncthreads();
    }
    if (tid == 0) fail[cand] = 0;
}

// (Y, dY) of every storage block as a 64 x 32 column-major tile of pairs (zeros
// outside the panel and on its padding slots, which start from zero; dY == nullptr
// gives dy = 0): the one-wave factorisation reads a panel row per lane, each load
// one column of 64 consecutive pairs.
__global__ void __launch_bounds__(256)
k_yd_rows(const int *__restrict__ bl_first, const int64_t *__restrict__ bl_rptr, const int64_t *__restrict__ bl_off,
          const double *__restrict__ wE, const double *__restrict__ Y, const double *__restrict__ dY,
          double2 *__restrict__ yd) {
    const int b = blockIdx.x;
    const int w = bl_first[b + 1] - bl_first[b];
    const int h = int(bl_rptr[b + 1] - bl_rptr[b]);
    const int64_t off = bl_off[b];
    for (int e = threadIdx.x; e < 64 * 32; e += blockDim.x) {
        const int i = e % 64, k = e / 64;
        double2 v = double2{0.0, 0.0};
        if (i < h && k < w) {
            const int64_t s = off + i + int64_t(h) * k;
            if (wE[s] != 0.0) v = double2{Y[s], dY ? dY[s] : 0.0};
        }
        yd[size_t(b) * 64 * 32 + e] = v;
    }
}

// Y = N N^T on the storage blocks by a single wave (panels of at most 64 rows and
// 32 columns).  Lane i holds row i of the panel in registers.  The elimination
// broadcasts the pivot and the next column's multiplier by readlane and the other
// multipliers through a 64-double LDS buffer (elim_lds).  The update of the
// ancestors, N(U, U) -= L21 L21^T, runs on the FP64 MFMA: L21 (at most 16 RT rows,
// row-major in LDS) is cut into RT row tiles and every lower tile pair is one
// chain of eight 16 x 16 x 4 products; wc_up gives, in the MFMA's lane order, the
// pending-update slot code of each result element (-1 where there is none: above
// the diagonal, outside the structure, padding rows).
// blockIdx.x selects the candidate Y + alpha_c dY (dual == false: Y itself).  The
// candidate is never written out: a panel is formed when its block is reached,
// from Y and dY (copied per panel column by column by k_yd_rows, read one block ahead
// while the previous block is factorised) and the pending updates of its
// descendants.  Those live in slots; the second last (ustride - 2) stays zero and is
// read by the panel entries that receive no update (su_rows gives every entry's
// slot), the last takes the results that update nothing (so every lane writes); with POOL
// the slots are a pool in LDS, reused once a panel has consumed them, otherwise
// a per-candidate array in global memory.  The first update of a slot in block
// order overwrites it (code = slot << 1 | first), so no other slot needs clearing.  The
// factor is stored (the whole panel, zeros above the diagonal) only by the
// candidates whose factor is used afterwards: the gamma twins, or the single
// factorisation when dual is false.  The block sizes (wc_meta: w, h, offset) come
// with the block's other inputs, one block ahead, through vector loads.
constexpr int kPrLd = 34;      // LDS row stride of L21 (doubles): rows fall on different banks
typedef double wd4 __attribute__((ext_vector_type(4)));   // one MFMA accumulator

template <bool POOL, int RT>
__global__ void __launch_bounds__(64)
k_sn_chol_wave(int nb, const int *__restrict__ wc_meta, const int4 *__restrict__ wc_up,
               const int *__restrict__ su_rows, const double2 *__restrict__ yd_rows, bool dual,
               const double *__restrict__ bracket, int round, int ntest, double gamma,
               double *__restrict__ Lbase, int64_t stride, double *__restrict__ Ubase, int64_t ustride,
               int prcap, int *__restrict__ fail) {
    constexpr int MT = RT * (RT + 1) / 2;   // lower tile pairs (ti >= tj), ti-major
    extern __shared__ double sm[];
    double *Pr = sm;            // rows of the factored panel, kPrLd doubles per row (prcap doubles)
    double *Wl = sm + prcap;    // the elimination's multipliers (64 doubles, 16-byte aligned)
    const int lane = threadIdx.x;
    const int cand = blockIdx.x;
    // each candidate is one long dependent chain: ahead of the waves of concurrent kernels
    __builtin_amdgcn_s_setprio(3);
    if (dual && round > 0 && bracket[2] != 0.0) {   // settled: nothing to test
        if (lane == 0) fail[cand] = 0;
        return;
    }
    const double al = dual ? cand_alpha(cand, ntest, round, gamma, bracket) : 0.0;
    const bool keep = !dual || cand >= ntest;   // the factor is used afterwards
    double *L = Lbase + cand * stride;
    double *U = POOL ? sm + prcap + 64 : Ubase + cand * ustride;
    if (lane == 0) U[ustride - 2] = 0.0;   // the slot of the entries without updates
    if (!POOL) __threadfence_block();
    // inputs of the next block, in flight while the current block is processed: the
    // row lane of its 64 x 32 tile (32 (y, dy) pairs and 32 slot codes; each load
    // reads one column, or four columns of codes, for all 64 rows), its sizes and its
    // update codes
    double2 q[32];
    int qsu[32];
    int qm;
    int4 qu[MT];
    auto issue = [&](int bb) {
        const double2 *yp = yd_rows + size_t(bb) * 2048 + lane;
        const int4 *sp = reinterpret_cast<const int4 *>(su_rows) + size_t(bb) * 512 + lane;
#pragma unroll
        for (int k = 0; k < 32; ++k) q[k] = yp[64 * k];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int4 t = sp[64 * u];
            qsu[4 * u] = t.x;
            qsu[4 * u + 1] = t.y;
            qsu[4 * u + 2] = t.z;
            qsu[4 * u + 3] = t.w;
        }
        qm = wc_meta[4 * bb + (lane & 3)];
#pragma unroll
        for (int t = 0; t < MT; ++t) qu[t] = wc_up[(size_t(bb) * MT + t) * 64 + lane];
    };
    issue(0);
    for (int b = 0; b < nb; ++b) {
        const int w = __builtin_amdgcn_readlane(qm, 0);
        const int h = __builtin_amdgcn_readlane(qm, 1);
        const int64_t off = __builtin_amdgcn_readlane(qm, 2);
        const int hp = h - w;
        int4 up[MT];
#pragma unroll
        for (int t = 0; t < MT; ++t) up[t] = qu[t];
        // the panel of the candidate: Y + alpha dY plus the pending updates
        double a[32];
        int su[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            a[k] = fma(al, q[k].y, q[k].x);
            su[k] = qsu[k];
        }
        if (b + 1 < nb) issue(b + 1);
#pragma unroll
        for (int k = 0; k < 32; ++k) a[k] += U[su[k]];
        // 16 or 32 columns are eliminated: the columns k >= w only collect values that
        // nothing reads, and never feed the columns below w
        if (w <= 16) elim_lds<16>(reinterpret_cast<double(&)[16]>(a), 0, Wl);
        else elim_lds<32>(a, 0, Wl);
        // every row to LDS, columns >= w as zeros (rows >= h are zero): the diagonal for
        // the check below and, from row w on, the MFMA operands (prcap holds the rows up
        // to the largest h and w + 31)
        if (lane * kPrLd < prcap) {
            double2 *pr = reinterpret_cast<double2 *>(Pr + lane * kPrLd);
            if (w == 32) {   // uniform
#pragma unroll
                for (int k = 0; k < 32; k += 2) pr[k / 2] = double2{a[k], a[k + 1]};
            } else {
#pragma unroll
                for (int k = 0; k < 32; k += 2) pr[k / 2] = double2{k < w ? a[k] : 0.0, k + 1 < w ? a[k + 1] : 0.0};
            }
        }
        // a pivot that is not positive and finite leaves a NaN (or 0 * inf) on the
        // diagonal: one check per block instead of one per pivot inside the chain
        const double dg = Pr[min(lane, 31) * (kPrLd + 1)];
        if (__ballot(lane < w && !((dg > 0.0) && isfinite(dg))) != 0ull) {
            if (lane == 0) fail[cand] = b + 1;
            return;   // uniform
        }
        // the elimination left zeros above the diagonal, and rows >= h are zero
        if (keep && lane < h) {
            double *p = L + off + lane;
#pragma unroll
            for (int k = 0; k < 32; ++k) {
                if (k < w) *p = a[k];   // uniform
                p += h;
            }
        }
        // MFMA operands: lane l holds L21(16 t + l % 16, 4 s + l / 16), zero below row hp
        // (with two row tiles the rows read are below 64 and zero beyond h)
        double x[RT][8];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const int row = 16 * t + (lane & 15);
            const double *pr = Pr + (w + (RT == 2 ? row : max(min(row, hp - 1), 0))) * kPrLd + (lane >> 4);
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const double v = pr[4 * s];
                x[t][s] = (RT == 2 || row < hp) ? v : 0.0;
            }
        }
        // element r of tile pair t: L21 L21^T(16 ti + 4 r + l / 16, 16 tj + l % 16)
        auto apply = [&](const int4 &c, const wd4 &v) {
            U[c.x >> 1] = ((c.x & 1) ? 0.0 : U[c.x >> 1]) - v[0];
            U[c.y >> 1] = ((c.y & 1) ? 0.0 : U[c.y >> 1]) - v[1];
            U[c.z >> 1] = ((c.z & 1) ? 0.0 : U[c.z >> 1]) - v[2];
            U[c.w >> 1] = ((c.w & 1) ? 0.0 : U[c.w >> 1]) - v[3];
        };
        // all tile pairs' chains interleaved; with four row tiles, one row tile's
        // pairs at a time (registers)
        constexpr int G = RT <= 2 ? RT : 1;   // row tiles per group
#pragma unroll
        for (int g = 0; g < RT; g += G) {
            constexpr int NG = G == RT ? MT : RT;   // most pairs in a group
            wd4 acc[NG];
#pragma unroll
            for (int t = 0; t < NG; ++t) acc[t] = wd4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                int t = 0;
#pragma unroll
                for (int ti = g; ti < g + G; ++ti)
#pragma unroll
                    for (int tj = 0; tj <= ti; ++tj, ++t)
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[ti][s], x[tj][s], acc[t], 0, 0, 0);
            }
            int t = 0;
#pragma unroll
            for (int ti = g; ti < g + G; ++ti)
#pragma unroll
                for (int tj = 0; tj <= ti; ++tj, ++t) apply(up[ti * (ti + 1) / 2 + tj], acc[t]);
        }
        // the next block reads these updates (other lanes' included)
        if (POOL) __builtin_amdgcn_s_waitcnt(0xc07f);
        else __threadfence_block();
        __builtin_amdgcn_wave_barrier();
    }
    if (lane == 0) fail[cand] = 0;
}

__global__ void __launch_bounds__(64)
k_dinv(const int *__restrict__ bl_first, const int64_t *__restrict__ bl_rptr, const int64_t *__restrict__ bl_off,
       const int64_t *__restrict__ bl_dinv, const double *__restrict__ L, double *__restrict__ Dinv,
       int *__restrict__ fail, double *__restrict__ G, const double *__restrict__ Dm) {
    __shared__ double D[64 * 64];
    const int b = blockIdx.x;
    const int F = bl_first[b];
    const int w = bl_first[b + 1] - F;
    const int h = int(bl_rptr[b + 1] - bl_rptr[b]);
    const double *P = L + bl_off[b];
    for (int i = threadIdx.x; i < w * w; i += blockDim.x) {
        const int r = i % w, c = i / w;
        D[i] = (r >= c) ? P[r + int64_t(h) * c] : 0.0;
    }
    __syncthreads();
    double *X = Dinv + bl_dinv[b];
    const int k = threadIdx.x;
    // column k of D^{-1} by forward substitution, in registers (w <= 32: loops of fixed
    // length, rows beyond w skipped uniformly; the terms j < k add exact zeros)
    double xs[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) xs[i] = 0.0;
    if (k < w) {
        const double dk = D[k + w * k];
        if (!(dk != 0.0) || !isfinite(dk)) atomicExch(fail, b + 1);
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            if (i < w) {   // uniform
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < i; ++j) acc += D[i + w * j] * xs[j];
                xs[i] = (i == k) ? 1.0 / dk : ((i > k) ? -acc / D[i + w * i] : 0.0);
            }
        }
#pragma unroll
        for (int i = 0; i < 32; ++i)
            if (i < w) X[i + w * k] = xs[i];
    }
    if (G && w <= 32 && h <= 64) {
        // G_b = [D^{-1}; P21 D^{-1}] (h x w): D^{-1} (each thread its column), P21 and G
        // in LDS over D (w h <= 2048 doubles each part), D^{-1}(j, c) = 0 for j < c;
        // then stored in the walks' lane order, zero outside the block:
        //   forward  (wave f < 4, lane l, ks < 8):  G(16 f + l % 16, 4 ks + l / 16)
        //   backward (wave f < 2, lane l, ks < 16): G(4 ks + l / 16, 16 f + l % 16)
        // With Dm the forward operand's top block is Dm_b D^{-1} (in LDS where P21 was).
        __syncthreads();
        double *Xs = D, *Ps = D + w * w, *Gs = D + 2048;
        const int hw = h - w;
        if (k < w) {
#pragma unroll
            for (int i = 0; i < 32; ++i)
                if (i < w) Xs[i + w * k] = xs[i];
        }
        for (int i = threadIdx.x; i < hw * w; i += blockDim.x) Ps[i] = P[(w + i % hw) + int64_t(h) * (i / hw)];
        __syncthreads();
        for (int i = threadIdx.x; i < h * w; i += blockDim.x) {
            const int r = i % h, c = i / h;
            double acc = 0.0;
            if (r < w) {
                acc = Xs[r + w * c];
            } else {
                for (int j = c; j < w; ++j) acc = fma(Ps[(r - w) + hw * j], Xs[j + w * c], acc);
            }
            Gs[r + h * c] = acc;
        }
        __syncthreads();
        double *Ts = Ps;   // w x w, after P21 is no longer read (w w <= 2048 - w w)
        if (Dm) {
            const double *Db = Dm + bl_dinv[b];
            for (int i = threadIdx.x; i < w * w; i += blockDim.x) {
                const int r = i % w, c = i / w;
                double acc = 0.0;
                for (int j = c; j < w; ++j) acc = fma(Db[r + w * j], Xs[j + w * c], acc);
                Ts[i] = acc;
            }
            __syncthreads();
        }
        double *Gb = G + size_t(b) * 4096;
        for (int i = threadIdx.x; i < 2048; i += blockDim.x) {
            const int ks = i % 8, l = (i / 8) % 64, f = i / 512;
            const int r = 16 * f + l % 16, c = 4 * ks + l / 16;
            Gb[i] = (r < h && c < w) ? ((Dm && r < w) ? Ts[r + w * c] : Gs[r + h * c]) : 0.0;
        }
        for (int i = threadIdx.x; i < 2048; i += blockDim.x) {
            const int ks = i % 16, l = (i / 16) % 64, f = i / 1024;
            const int r = 4 * ks + l / 16, c = 16 * f + l % 16;
            Gb[2048 + i] = (r < h && c < w) ? Gs[r + h * c] : 0.0;
        }
    }
}

__global__ void __launch_bounds__(256)
k_algorithm1(const int64_t *__restrict__ cl_ptr, const int64_t *__restrict__ cl_map_ptr,
             const int *__restrict__ cl_map, const int *__restrict__ cl_first, const double *__restrict__ Xbar,
             double *__restrict__ Lhat, int *__restrict__ fail) {
    __shared__ TileLds<64, 64> sh;
    const int r = blockIdx.x;
    const int c = int(cl_ptr[r + 1] - cl_ptr[r]);
    const int ns = cl_first[r + 1] - cl_first[r];
    const int *map = cl_map + cl_map_ptr[r];
    const int tid = threadIdx.x;
    const int i0 = 4 * (tid / 16), j0 = 4 * (tid % 16);
    // packed lower index of clique entry (ii, jj), ii >= jj: jj * (2c - jj + 1) / 2 + (ii - jj)
    auto pk = [c](int ii, int jj) { return jj * (2 * c - jj + 1) / 2 + (ii - jj); };
    // Z = P_r Xbar(C_r, C_r) P_r^T, Z(a, b) = Xbar(C[c-1-a], C[c-1-b]);
    // identity beyond the clique order
    double a[4][4], m[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + u, k = j0 + v;
            a[u][v] = (i < c && k <= i) ? Xbar[map[pk(c - 1 - k, c - 1 - i)]] : (i == k ? 1.0 : 0.0);
            m[u][v] = (i == k) ? 1.0 : 0.0;
        }
    // Z = M_r M_r^T, with M_r^{-1} alongside
    int bad = 0;
    if (!chol_tile<4, 4, 16, true>(a, m, c, sh, &bad)) {
        if (tid == 0) atomicCAS(fail, 0, r + 1);
        return;
    }
    // L_r = P_r M_r^{-T} P_r^T, i.e. L_r(ii, jj) = M_r^{-1}(c-1-jj, c-1-ii); its first
    // ns columns are Lhat(C_r, S_r), i.e. rows >= c - ns of M_r^{-1}
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + u, k = j0 + v;
            if (i < c && i >= c - ns && k <= i) Lhat[map[pk(c - 1 - k, c - 1 - i)]] = m[u][v];
        }
}

// The earlier factorisation X^ = L^T D L (eqs. sparse_fact, orig_L, orig_D of
// Section 2.1), per clique C_r = S_r + U_r: the block in the order [U_r; S_r],
// Z = [[X_UU, X_US], [X_SU, X_SS]], is eliminated over its first |U_r| columns
// only.  That leaves the Schur complement X_SS - X_SU X_UU^{-1} X_US = D_r in the
// trailing block, and the partially eliminated identity E = [[R^{-1}, 0],
// [-X_SU X_UU^{-1}, I]] (X_UU = R R^T), whose lower-left block is the transpose
// of the (U_r, S_r) block of L^{-1} = I - sum_r (L_r - I).  L^{-1}
// (unit lower, on E, rows C_r x columns S_r) goes into the factor layout, D_r into
// the w x w diagonal-block array of the storage block holding S_r (zero between
// supernodes).  A second elimination of all |C_r| columns checks that D_r (hence
// Xbar(C_r, C_r)) is positive definite.
__global__ void __launch_bounds__(256)
k_ldl_clique(const int64_t *__restrict__ cl_ptr, const int64_t *__restrict__ cl_map_ptr,
             const int *__restrict__ cl_map, const int *__restrict__ cl_first, const int *__restrict__ col_block,
             const int *__restrict__ bl_first, const int64_t *__restrict__ bl_dinv,
             const double *__restrict__ Xbar, double *__restrict__ Linv, double *__restrict__ Dblk,
             int *__restrict__ fail) {
    __shared__ TileLds<64, 64> sh;
    const int r = blockIdx.x;
    const int c = int(cl_ptr[r + 1] - cl_ptr[r]);
    const int ns = cl_first[r + 1] - cl_first[r];
    const int nu = c - ns;
    const int *map = cl_map + cl_map_ptr[r];
    const int tid = threadIdx.x;
    const int i0 = 4 * (tid / 16), j0 = 4 * (tid % 16);
    auto pk = [c](int ii, int jj) { return jj * (2 * c - jj + 1) / 2 + (ii - jj); };
    // Z index -> clique member: U first, then S
    auto mem = [ns, nu](int z) { return z < nu ? ns + z : z - nu; };
    auto xval = [&](int za, int zb) {   // Xbar(member(za), member(zb))
        int ii = mem(za), jj = mem(zb);
        if (ii < jj) { const int t = ii; ii = jj; jj = t; }
        return Xbar[map[pk(ii, jj)]];
    };
    double a[4][4], e[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + u, k = j0 + v;
            a[u][v] = (i < c && k <= i) ? xval(i, k) : (i == k ? 1.0 : 0.0);
            e[u][v] = (i == k) ? 1.0 : 0.0;
        }
    int bad = 0;
    if (!chol_tile<4, 4, 16, true>(a, e, nu, sh, &bad)) {
        if (tid == 0) atomicCAS(fail, 0, r + 1);
        return;
    }
    // D_r: the trailing block (lower triangle valid), stored symmetric
    const int F = cl_first[r], b = col_block[F], Fb = bl_first[b], w = bl_first[b + 1] - Fb;
    double *Db = Dblk + bl_dinv[b];
    const int s0 = F - Fb;   // first column of S_r inside the storage block
    double dkeep[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + u, k = j0 + v;
            dkeep[u][v] = a[u][v];
            if (i < c && k <= i && k >= nu) {
                const int si = i - nu, sk = k - nu;
                Db[(s0 + si) + w * (s0 + sk)] = a[u][v];
                Db[(s0 + sk) + w * (s0 + si)] = a[u][v];
            }
            // (U_r, S_r) block of L^{-1}: Linv(member ns + k, member i - nu) = E(i, k)
            if (i < c && i >= nu && k < nu) Linv[map[pk(ns + k, i - nu)]] = e[u][v];
        }
    for (int t = tid; t < ns * (ns + 1) / 2; t += blockDim.x) {   // S_r x S_r block: the identity
        int jj = 0, rem = t;
        while (rem >= ns - jj) { rem -= ns - jj; ++jj; }
        const int ii = jj + rem;
        Linv[map[pk(ii, jj)]] = (ii == jj) ? 1.0 : 0.0;
    }
    // D_r positive definite: eliminate it on its own (identity in the U rows)
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + u, k = j0 + v;
            a[u][v] = (i < c && k <= i && k >= nu) ? dkeep[u][v] : (i == k ? 1.0 : 0.0);
        }
    if (!chol_tile<4, 4, 16, false>(a, e, c, sh, &bad))
        if (tid == 0) atomicCAS(fail, 0, r + 1);
}

__global__ void __launch_bounds__(256)
k_alpha_cl(const int64_t *__restrict__ cl_ptr, const int64_t *__restrict__ cl_map_ptr,
           const int *__restrict__ cl_map, const double *__restrict__ Xbar, const double *__restrict__ dX,
           double *__restrict__ alpha_cl) {
    __shared__ TileLds<64, 64> sh;
    const int r = blockIdx.x;
    const int c = int(cl_ptr[r + 1] - cl_ptr[r]);
    const int *map = cl_map + cl_map_ptr[r];
    const int tid = threadIdx.x;
    const int i0 = 4 * (tid / 16), j0 = 4 * (tid % 16);
    auto pk = [c](int ii, int jj) { return jj * (2 * c - jj + 1) / 2 + (ii - jj); };
    // the clique block in the reversed order Algorithm 1 factorises in; identity
    // (and a zero direction) beyond the clique order
    double x[4][4], dx[4][4], a[4][4], unused[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + u, k = j0 + v;
            const bool in = i < c && k <= i;
            const int s = in ? map[pk(c - 1 - k, c - 1 - i)] : 0;
            x[u][v] = in ? Xbar[s] : (i == k ? 1.0 : 0.0);
            dx[u][v] = in ? dX[s] : 0.0;
            unused[u][v] = 0.0;
        }
    auto test = [&](double al) -> bool {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) a[u][v] = fma(al, dx[u][v], x[u][v]);
        int bad = 0;
        return chol_tile<4, 4, 16, false>(a, unused, c, sh, &bad);
    };
    double res;
    if (test(1.0)) {
        res = 1.0;
    } else {
        double lo = 0.0, hi = 1.0;
        for (int it = 0; it < 52; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            if (test(mid)) lo = mid; else hi = mid;
        }
        res = lo;
    }
    if (tid == 0) alpha_cl[r] = res;
}

// The same step lengths for cliques of at most 32 members, one wave per clique (four
// per workgroup) and no barriers: lane i holds row i of the clique block (in the
// reversed order Algorithm 1 factorises in) and of the direction; each test is a
// readlane elimination as in k_sn_chol_wave, a pivot that is not positive and
// finite leaving a NaN on the diagonal.  The bisection is the same, run in two
// launches: phase 0 tests 1 and takes the first `steps` halvings of (0, 1),
// leaving (lo, hi) per clique; phase 1 finishes the bisection only for the cliques
// whose lo is below the smallest hi (*mhi), the only ones whose result can be the
// minimum over the cliques; the others keep lo, no smaller than that minimum.  The
// minimum is the one the whole bisection of every clique gives.
__global__ void __launch_bounds__(256)
k_alpha_cl_wave(int ncl, const int64_t *__restrict__ cl_ptr, const int64_t *__restrict__ cl_map_ptr,
                const int *__restrict__ cl_map, const double *__restrict__ Xbar, const double *__restrict__ dX,
                double *__restrict__ alpha_lo, double *__restrict__ alpha_hi, int phase, int steps,
                const double *__restrict__ mhi) {
    const int r = 4 * int(blockIdx.x) + int(threadIdx.x >> 6);
    if (r >= ncl) return;   // uniform per wave
    double lo = 0.0, hi = 1.0;
    if (phase == 1) {
        lo = alpha_lo[r];
        hi = alpha_hi[r];
        if (!(lo < *mhi)) return;   // uniform: not a candidate for the minimum
    }
    const int lane = threadIdx.x & 63;
    const int c = int(cl_ptr[r + 1] - cl_ptr[r]);
    const int *map = cl_map + cl_map_ptr[r];
    auto pk = [c](int ii, int jj) { return jj * (2 * c - jj + 1) / 2 + (ii - jj); };
    double x[32], dx[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        const bool in = lane < c && k <= lane;
        const int sl = in ? map[pk(c - 1 - k, c - 1 - lane)] : 0;
        x[k] = in ? Xbar[sl] : (lane == k ? 1.0 : 0.0);
        dx[k] = in ? dX[sl] : 0.0;
    }
    auto test = [&](double al) -> bool {
        double a[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) a[k] = fma(al, dx[k], x[k]);
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            if (k < c) {   // uniform
                const double d = lane_bcast(a[k], k);
                const double inv = rsqrt_newton(d);
                const double l = (lane >= k) ? a[k] * inv : 0.0;
                a[k] = l;
                elim_step_bcast(a, l, k, 0);
            }
        }
        double dg = 0.0;
#pragma unroll
        for (int k = 0; k < 32; ++k)
            if (k == lane) dg = a[k];
        return __ballot(lane < c && !((dg > 0.0) && isfinite(dg))) == 0ull;
    };
    if (phase == 0 && test(1.0)) {
        lo = hi = 1.0;
    } else {
        for (int it = 0; it < steps; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            if (test(mid)) lo = mid; else hi = mid;
        }
    }
    if (lane == 0) {
        alpha_lo[r] = lo;
        alpha_hi[r] = hi;
    }
}

// After a round of candidate tests (fail[c] == 0: Y + a_c dY positive definite),
// keep the longest prefix of successful test points and narrow
// bracket = (lo, hi, settled, twin): twin is the candidate index holding the
// factor of Y + gamma lo dY, or -1 if that factor was not formed.
__global__ void __launch_bounds__(1024) k_bracket(int ntest, int round, int twins, double gamma,
                                                   const int *__restrict__ fail, double *__restrict__ bracket) {
    __shared__ int first;   // first test point that failed (ntest if none)
    if (round > 0 && bracket[2] != 0.0) return;   // uniform: settled
    if (threadIdx.x == 0) first = ntest;
    __syncthreads();
    for (int c = threadIdx.x; c < ntest; c += blockDim.x)
        if (fail[c] != 0) atomicMin(&first, c);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int best = first - 1;   // the longest prefix of test points that passed
    auto cand = [&](int c) { return cand_alpha(c, ntest, round, gamma, bracket); };
    if (round == 0) {
        if (best == ntest - 1) {   // alpha = 1 passes; its twin (candidate ntest) is gamma * 1
            bracket[0] = 1.0; bracket[1] = 1.0; bracket[2] = 1.0;
            bracket[3] = (fail[ntest] == 0) ? double(ntest) : -1.0;
            return;
        }
        // no grid point passed: the step is below the grid's smallest point, and the
        // next round searches (0, that point) evenly instead of giving up
        if (best < 0) { bracket[0] = 0.0; bracket[1] = cand(0); bracket[2] = 0.0; bracket[3] = -1.0; return; }
        const double lo = cand(best), hi = cand(best + 1);
        bracket[0] = lo; bracket[1] = hi; bracket[2] = 0.0; bracket[3] = -1.0;
        return;
    }
    const double lo = best >= 0 ? cand(best) : bracket[0];
    const double hi = best + 1 < ntest ? cand(best + 1) : bracket[1];
    const double twin = (twins && best >= 0 && fail[ntest + best] == 0) ? double(ntest + best) : -1.0;
    bracket[0] = lo;
    bracket[1] = hi;
    bracket[3] = twin;
}

__global__ void __launch_bounds__(1024) k_min_reduce(int len, const double *__restrict__ v, double *out) {
    __shared__ double sh[1024];
    double m = 1.0;
    for (int i = threadIdx.x; i < len; i += blockDim.x) m = fmin(m, v[i]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

}  // namespace

// LDS of the one-wave factorisation: the rows of L21, the multipliers and, with a
// pool, the pool
static size_t wave_chol_lds(const DevStruct &d) {
    return wave_chol_lds_bytes(d.max_h, d.max_w, d.u_pool ? d.nU : 0);
}

static void launch_wave_chol(const DevStruct &d, int nc, const double2 *yd, bool dual, const double *bracket,
                             int round, int ntest, double gamma, double *L, int64_t stride, double *U, int *fail,
                             hipStream_t st) {
    const int prcap = wave_chol_rows(d.max_h, d.max_w) * kPrLd;
    const int4 *up = reinterpret_cast<const int4 *>(d.wc_up);
#define SDPC_WAVE_CHOL(POOL, RT)                                                                                 \
    hipLaunchKernelGGL((k_sn_chol_wave<POOL, RT>), dim3(nc), dim3(64), wave_chol_lds(d), st, d.nb, d.wc_meta, up, \
                       d.su_rows, yd, dual, bracket, round, ntest, gamma, L, stride, U, d.nU, prcap, fail)
    if (d.wc_rt == 2) {
        if (d.u_pool) SDPC_WAVE_CHOL(true, 2);
        else SDPC_WAVE_CHOL(false, 2);
    } else {
        if (d.u_pool) SDPC_WAVE_CHOL(true, 4);
        else SDPC_WAVE_CHOL(false, 4);
    }
#undef SDPC_WAVE_CHOL
}

size_t wave_chol_work_doubles(const DevStruct &d) { return size_t(d.nb) * 64 * 32 * 2; }

int wave_chol_rows(int max_h, int max_w) { return std::min(64, std::max(max_h, max_w + 32)); }

size_t wave_chol_lds_bytes(int max_h, int max_w, int64_t npool) {
    return sizeof(double) * (size_t(wave_chol_rows(max_h, max_w)) * kPrLd + 64 + size_t(npool < 1 ? 1 : npool));
}

void launch_sn_chol(const DevStruct &d, const double *Y, double *L, double *U, double *work, int *fail,
                    hipStream_t st) {
    if (d.max_h <= 64) {
        double2 *yd = reinterpret_cast<double2 *>(work);
        hipLaunchKernelGGL(k_yd_rows, dim3(d.nb), dim3(256), 0, st, d.bl_first, d.bl_rptr, d.bl_off, d.wE, Y,
                           (const double *)nullptr, yd);
        launch_wave_chol(d, 1, yd, false, nullptr, 0, 1, 0.0, L, 0, U, fail, st);
        return;
    }
    const size_t lds = size_t(d.max_panel) * sizeof(double);
    hipLaunchKernelGGL(k_sn_chol, dim3(1), dim3(kCholThreads), lds, st, d.nb, d.nslot, d.wE, d.bl_first,
                       d.bl_rptr, d.bl_off, d.up_ptr, d.up_pair, d.up_slot, Y, (const double *)nullptr,
                       (const double *)nullptr, 0, 1, 0.0, L, int64_t(0), fail);
}

// round 0: its test points and the twin of alpha = 1; later rounds: their test points,
// and in the last round one twin per test point (the twin of the step finally taken)
int dual_step_candidates(int round, int rounds, const int *ntest) {
    return round == 0 ? ntest[0] + 1 : (round == rounds - 1 ? 2 * ntest[round] : ntest[round]);
}

void launch_dual_step(const DevStruct &d, const double *Y, const double *dY, int rounds, const int *ntest,
                      double gamma, double *cand, double *U, double *work, int *fail, double *bracket,
                      hipStream_t st) {
    const size_t lds = size_t(d.max_panel) * sizeof(double);
    double2 *yd = reinterpret_cast<double2 *>(work);
    if (d.max_h <= 64)
        hipLaunchKernelGGL(k_yd_rows, dim3(d.nb), dim3(256), 0, st, d.bl_first, d.bl_rptr, d.bl_off, d.wE, Y, dY,
                           yd);
    for (int r = 0; r < rounds; ++r) {
        const int nc = dual_step_candidates(r, rounds, ntest);
        if (d.max_h <= 64) {
            launch_wave_chol(d, nc, yd, true, bracket, r, ntest[r], gamma, cand, d.nslot, U, fail, st);
        } else {
            hipLaunchKernelGGL(k_sn_chol, dim3(nc), dim3(kCholThreads), lds, st, d.nb, d.nslot, d.wE, d.bl_first,
                               d.bl_rptr, d.bl_off, d.up_ptr, d.up_pair, d.up_slot, Y, dY, (const double *)bracket,
                               r, ntest[r], gamma, cand, d.nslot, fail);
        }
        hipLaunchKernelGGL(k_bracket, dim3(1), dim3(1024), 0, st, ntest[r], r, (r > 0 && r == rounds - 1) ? 1 : 0,
                           gamma, (const int *)fail, bracket);
    }
}

void launch_dinv(const DevStruct &d, const double *L, double *Dinv, int *fail, hipStream_t st, double *G,
                 const double *Dm) {
    hipLaunchKernelGGL(k_dinv, dim3(d.nb), dim3(64), 0, st, d.bl_first, d.bl_rptr, d.bl_off, d.bl_dinv, L,
                       Dinv, fail, G, Dm);
}

void launch_algorithm1(const DevStruct &d, const double *Xbar, double *Lhat, int *fail, hipStream_t st) {
    hipLaunchKernelGGL(k_algorithm1, dim3(d.ncl), dim3(256), 0, st, d.cl_ptr, d.cl_map_ptr, d.cl_map,
                       d.cl_first, Xbar, Lhat, fail);
}

void launch_ldl_cliques(const DevStruct &d, const double *Xbar, double *Linv, double *Dblk, int *fail,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_ldl_clique, dim3(d.ncl), dim3(256), 0, st, d.cl_ptr, d.cl_map_ptr, d.cl_map, d.cl_first,
                       d.col_block, d.bl_first, d.bl_dinv, Xbar, Linv, Dblk, fail);
}

void launch_alpha_cliques(const DevStruct &d, const double *Xbar, const double *dX, double *alpha_cl,
                          double *alpha_hi, double *out, hipStream_t st) {
    if (d.max_clique <= 32) {
        // 52 halvings in all: 10 for every clique, the rest for the candidates
        constexpr int kFirst = 10;
        hipLaunchKernelGGL(k_alpha_cl_wave, dim3((d.ncl + 3) / 4), dim3(256), 0, st, d.ncl, d.cl_ptr, d.cl_map_ptr,
                           d.cl_map, Xbar, dX, alpha_cl, alpha_hi, 0, kFirst, (const double *)nullptr);
        hipLaunchKernelGGL(k_min_reduce, dim3(1), dim3(1024), 0, st, d.ncl, (const double *)alpha_hi, out);
        hipLaunchKernelGGL(k_alpha_cl_wave, dim3((d.ncl + 3) / 4), dim3(256), 0, st, d.ncl, d.cl_ptr, d.cl_map_ptr,
                           d.cl_map, Xbar, dX, alpha_cl, alpha_hi, 1, 52 - kFirst, (const double *)out);
    } else {
        hipLaunchKernelGGL(k_alpha_cl, dim3(d.ncl), dim3(256), 0, st, d.cl_ptr, d.cl_map_ptr, d.cl_map, Xbar, dX,
                           alpha_cl);
    }
    hipLaunchKernelGGL(k_min_reduce, dim3(1), dim3(1024), 0, st, d.ncl, (const double *)alpha_cl, out);
}

}  // namespace sdpc
