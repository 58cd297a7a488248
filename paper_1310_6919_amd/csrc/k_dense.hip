// Dense FP64 Cholesky of the Schur complement matrix, B = R R^T (type (i) of
// Section 3.1), and the backward substitution of the SCE (eq. SCE).
//
// Right-looking, 64-wide column blocks, one fused launch per block column s:
//   workgroups 0..nt-1   tile rows s .. of column block s.  Each applies the
//                        pending panel s-1 to the diagonal tile and factorises it
//                        in one wave (lane = row, pivot column broadcast with
//                        readlane).  Workgroup 0 stores R_ss and reports a failed
//                        pivot; every other one also applies panel s-1 to its own
//                        tile, forms R_ss^{-1} (block inverses, the off-diagonal
//                        block on the MFMA) and solves X R_ss^T = C as one MFMA
//                        product.  Repeating the small factorisation in every
//                        workgroup of the column spares a hand-over through
//                        memory on the critical path.
//   the others           apply panel s-1 to every lower tile of the column blocks
//                        s+1 .. (the bulk of the trailing update), overlapping the
//                        diagonal factorisations of the same launch.
// So column block s+1 only lacks panel s when launch s+1 starts, and the launch
// boundary is the only grid-wide synchronisation.  Rows beyond m ride along:
// with the right-hand side g stored as row m, the sweep leaves R^{-1} g there
// (the forward substitution of the SCE), and only R^T x = R^{-1} g remains,
// done by one launch whose workgroups hand the blocks of x down through flags.
//
// Every wait of that solve is a bounded spin on a flag released by a workgroup
// with a lower index (dispatched earlier), so it cannot deadlock; a wait that
// runs out marks the call failed (fail = -1) instead of hanging.  Flags hold the
// epoch of the call that released them, so they never need to be cleared.
#include "chol_reg.h"
#include "kernels.h"

namespace sdpc {

namespace {

constexpr int NB = 64;
constexpr int LDS_LD = NB + 1;          // padded row length of a tile in LDS
constexpr int kSpinLimit = 1 << 20;     // about a second of polling before a wait gives up

typedef double d4 __attribute__((ext_vector_type(4)));

// One 64 x 64 output tile of C = A B^T (A, B column-major in global memory),
// operands loaded straight into registers in the FP64 16x16x4 MFMA layout.
// Operand layout of the MFMA D = X Z: lane l supplies X(l % 16, l / 16) and
// Z(l / 16, l % 16); element r of lane l's result is D(4 r + l / 16, l % 16)
// (checked on gfx950 with a lane-layout probe).  The product is formed as
// C^T = B A^T, so lane l, element r of acc[ti][tj] holds
//   C(qr + 16 ti + l % 16, qc + 16 tj + 4 r + l / 16),
// sixteen consecutive rows of one column per group of 16 lanes: operand loads
// and the write-back of a column-major C move whole 128-byte lines.  Each wave
// owns a 32 x 32 quadrant (qr, qc); all its operand loads are issued before the
// first product so one memory latency covers the whole tile.
struct TileIdx {
    int lane, li, lk, qr, qc;
    __device__ TileIdx() : TileIdx(int(threadIdx.x) / 64) {}
    __device__ explicit TileIdx(int quadrant) {   // quadrant w: rows 32 (w % 2), columns 32 (w / 2)
        lane = threadIdx.x % 64;
        li = lane % 16;
        lk = lane / 16;
        qr = 32 * (quadrant % 2);
        qc = 32 * (quadrant / 2);
    }
    __device__ int row(int ti) const { return qr + 16 * ti + li; }                 // tile row of acc[ti][.]
    __device__ int col(int tj, int r) const { return qc + 16 * tj + 4 * r + lk; }   // tile column of element r
};

// acc += A(ar0 + [0,64), ac0 + [0,kk)) * B(br0 + [0,64), bc0 + [0,kk))^T; rows of A at or
// beyond amax and rows of B at or beyond bmax read as zero; kk <= 64.
__device__ inline void tile_mma(const TileIdx &t, const double *A, int64_t lda, int ar0, int amax, int ac0,
                                const double *Bm, int64_t ldbm, int br0, int bmax, int bc0, int kk, d4 acc[2][2]) {
    double a[2][16], b[2][16];
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
        const int k = 4 * ks + t.lk;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int ra = ar0 + t.qr + 16 * u + t.li, rb = br0 + t.qc + 16 * u + t.li;
            a[u][ks] = (k < kk && ra < amax) ? A[ra + lda * (ac0 + k)] : 0.0;
            b[u][ks] = (k < kk && rb < bmax) ? Bm[rb + ldbm * (bc0 + k)] : 0.0;
        }
    }
#pragma unroll
    for (int ks = 0; ks < 16; ++ks)
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int tj = 0; tj < 2; ++tj)
                acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[tj][ks], a[ti][ks], acc[ti][tj], 0, 0, 0);
}

__device__ inline void zero_acc(d4 acc[2][2]) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
}

// Bounded wait for *flag == epoch (one thread); false if the wait ran out.
__device__ inline bool flag_wait(const int *flag, int epoch) {
    for (int it = 0; it < kSpinLimit; ++it) {
        if (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == epoch) return true;
        __builtin_amdgcn_s_sleep(2);
    }
    return false;
}

__device__ inline void flag_release(int *flag, int epoch) {
    __hip_atomic_store(flag, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Right-looking elimination of 32 columns held one row per lane (a[k] = A(lane,
// C0 + k)); pivot k sits in lane C0 + k and reaches the other lanes, with the
// scaled column, through readlane: no LDS, no barrier.  Lanes above the pivot get
// zero multipliers.  A pivot that is not positive and finite leaves a NaN on the
// diagonal of L (1/sqrt of it is NaN or makes 0 * inf), so the caller checks the
// diagonal afterwards instead of testing every pivot inside the chain.
template <int C0>
__device__ inline void panel32_wave(double (&a)[32]) {
    const int lane = threadIdx.x % 64;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        const double d = lane_bcast(a[k], C0 + k);
        const double inv = rsqrt_newton(d);
        const double l = (lane >= C0 + k) ? a[k] * inv : 0.0;   // row C0 + k gets sqrt(d)
        a[k] = l;
        elim_step_bcast(a, l, k, C0);
    }
}

// Cholesky of a 64 x 64 matrix held one row per lane by one wave, in two 32-column
// panels: lo[k] = A(lane, k), hi[k] = A(lane, 32 + k) (lower part used; the upper
// part ends meaningless).  Between the panels, A22 -= L21 L21^T is one 32 x 32 x 32
// product on the FP64 MFMA through the LDS scratch W (at least 32 x 33 + 32 x 33
// doubles).
__device__ inline void potrf64_wave(double (&lo)[32], double (&hi)[32], double *W) {
    const int lane = threadIdx.x % 64;
    panel32_wave<0>(lo);
    constexpr int LW = 33;
    double *D = W + 32 * LW;
    if (lane >= 32) {
#pragma unroll
        for (int k = 0; k < 32; ++k) W[(lane - 32) * LW + k] = lo[k];   // W = L21, row-major
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the wave's own LDS stores are done
    // D = W W^T, lower 16 x 16 blocks (0,0), (1,0), (1,1); lane l supplies
    // X(l % 16, l / 16) and Z(l / 16, l % 16); result element r: D(4 r + l / 16, l % 16)
    const int li = lane % 16, lk = lane / 16;
#pragma unroll
    for (int blk = 0; blk < 3; ++blk) {
        const int bi = (blk == 0) ? 0 : 1, bj = (blk == 2) ? 1 : 0;
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            const double x = W[(16 * bi + li) * LW + 4 * ks + lk];
            const double z = W[(16 * bj + li) * LW + 4 * ks + lk];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, z, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) D[(16 * bi + 4 * r + lk) * LW + 16 * bj + li] = acc[r];
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);
    if (lane >= 32) {
#pragma unroll
        for (int k = 0; k < 32; ++k)
            if (k <= lane - 32) hi[k] -= D[(lane - 32) * LW + k];
    }
    panel32_wave<32>(hi);
}

// The factor of diagonal block s (parked column-major in Rscr[s & 1]) into B:
// rows J0 + i < rows (right-hand-side rows riding along included), columns
// k < jb, k <= i.
__device__ inline void put_diag(double *B, int64_t ldb, int rows, int m, int s, const double *Rscr) {
    const int J0 = NB * s;
    const int jb = (m - J0 < NB) ? (m - J0) : NB;
    const double *Rs = Rscr + (s & 1) * NB * NB;
    for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
        const int i = idx % NB, k = idx / NB;
        if (J0 + i < rows && k < jb && k <= i) B[(J0 + i) + ldb * (J0 + k)] = Rs[idx];
    }
}

__global__ void __launch_bounds__(256)
k_put_diag(double *__restrict__ B, int64_t ldb, int rows, int m, int s, const double *__restrict__ Rscr) {
    put_diag(B, ldb, rows, m, s, Rscr);
}

__global__ void __launch_bounds__(256)
k_chol_step(double *__restrict__ B, int64_t ldb, int m, int rows, int s, int *__restrict__ fail,
            double *__restrict__ Rscr) {
    __shared__ double S[NB * LDS_LD];   // the updated tile, row-major; then the diagonal factor
    __shared__ double Ai[32 * 33], Ci[32 * 33], Eb[32 * 33];   // blocks of the factor's inverse
    __shared__ double invd[NB];
    const int tid = threadIdx.x;
    const TileIdx t;
    const int T_rows = (rows + NB - 1) / NB, T_cols = (m + NB - 1) / NB;
    const int nt = T_rows - s;
    const int J0 = NB * s;
    const int jb = (m - J0 < NB) ? (m - J0) : NB;
    if (int(blockIdx.x) >= nt) {
        // bulk: panel s-1 applied to the lower tile (I, K), s+1 <= K <= I
        int q = int(blockIdx.x) - nt, K = s + 1;
        while (K < T_cols && q >= T_rows - K) {
            q -= T_rows - K;
            ++K;
        }
        if (K >= T_cols) return;
        const int I = K + q;
        const int I0 = NB * I, K0 = NB * K, P0 = J0 - NB;
        double c[2][2][4];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gi = I0 + t.row(a), gk = K0 + t.col(b, r);
                    c[a][b][r] = (gi < rows && gk < m && gi >= gk) ? B[gi + ldb * gk] : 0.0;
                }
        d4 acc[2][2];
        zero_acc(acc);
        tile_mma(t, B, ldb, I0, rows, P0, B, ldb, K0, m, P0, NB, acc);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gi = I0 + t.row(a), gk = K0 + t.col(b, r);
                    if (gi < rows && gk < m && gi >= gk) B[gi + ldb * gk] = c[a][b][r] - acc[a][b][r];
                }
        return;
    }
    // column block s, tile row I.  Every workgroup of the column block factorises the
    // diagonal tile R_ss itself: a panel tile needs R_ss^{-1}, which it then forms in
    // its own LDS, so no workgroup waits on another; the diagonal workgroup alone
    // reports a failed pivot and stores R_ss.
    const int I = s + int(blockIdx.x), I0 = NB * I;
    const bool diag = (I == s);
    // quadrant tq of a tile of column block s with panel s-1 applied, in the
    // accumulator layout
    auto stage = [&](const TileIdx &tq, int R0, bool lower, double (&c)[2][2][4]) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gi = R0 + tq.row(a), gk = tq.col(b, r);
                    c[a][b][r] = (gi < rows && gk < jb && (!lower || gi >= J0 + gk)) ? B[gi + ldb * (J0 + gk)] : 0.0;
                }
        if (s >= 1) {
            d4 acc[2][2];
            zero_acc(acc);
            tile_mma(tq, B, ldb, R0, rows, J0 - NB, B, ldb, J0, m, J0 - NB, NB, acc);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) c[a][b][r] -= acc[a][b][r];
        }
    };
    auto to_lds = [&](const TileIdx &tq, const double (&c)[2][2][4]) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) S[tq.row(a) * LDS_LD + tq.col(b, r)] = c[a][b][r];
    };
    // the updated panel tile (I, s) is formed by waves 1..3 while wave 0 factorises the
    // diagonal tile, and parked in its own place in B until S is free again; each
    // thread reads back exactly the entries it wrote
    auto own_rw = [&](const TileIdx &tq, double (&c)[2][2][4], bool put) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gi = I0 + tq.row(a), gk = tq.col(b, r);
                    const bool in = gi < rows && gk < jb;
                    if (put) {
                        if (in) B[gi + ldb * (J0 + gk)] = c[a][b][r];
                    } else {
                        c[a][b][r] = in ? B[gi + ldb * (J0 + gk)] : 0.0;
                    }
                }
    };
    const int wv = tid >> 6;
    // quadrants of the panel tile: waves 1..3 their own, wave 1 also quadrant 0
    {
        double cd[2][2][4];
        stage(t, J0, true, cd);
        to_lds(t, cd);
    }
    __syncthreads();
    if (tid >= 64 && !diag) {
        double co[2][2][4];
        stage(t, I0, false, co);
        own_rw(t, co, true);
        if (wv == 1) {
            const TileIdx t0(0);
            stage(t0, I0, false, co);
            own_rw(t0, co, true);
        }
    }
    if (tid < 64) {
        __builtin_amdgcn_s_setprio(3);   // the chain of the launch: ahead of the bulk waves on this CU
        // rows of the tile below the block's own jb rows (right-hand-side rows riding
        // along the last block) keep their values in the jb active columns: the
        // elimination then performs their forward substitution
        const int lane = tid;
        const bool real = J0 + lane < rows;
        double lo[32], hi[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) {   // every load is in bounds; selects afterwards
            const double v0 = S[lane * LDS_LD + k], v1 = S[lane * LDS_LD + 32 + k];
            const int k2 = 32 + k;
            lo[k] = (real && k < jb) ? (k <= lane ? v0 : 0.0) : (lane == k ? 1.0 : 0.0);
            hi[k] = (real && k2 < jb) ? (k2 <= lane ? v1 : 0.0) : (lane == k2 ? 1.0 : 0.0);
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);   // the tile is in registers before S is reused
        potrf64_wave(lo, hi, S);               // S serves as its scratch
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            S[lane * LDS_LD + k] = lo[k];
            S[lane * LDS_LD + 32 + k] = hi[k];
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        const double dg = S[lane * LDS_LD + lane];
        if (diag) {
            // every pivot of the block must have been positive and finite
            const unsigned long long badm = __ballot(lane < jb && !((dg > 0.0) && isfinite(dg)));
            if (badm != 0ull && lane == 0) atomicCAS(fail, 0, J0 + __ffsll((long long)badm));
        } else {
            invd[lane] = 1.0 / dg;
            __builtin_amdgcn_s_waitcnt(0xc07f);
            // inverses of the four 16 x 16 diagonal blocks of R_ss: lane 16 g + j forms
            // column j of block g by forward substitution (four partial sums per row);
            // rows beyond the block's jb rows are taken as identity rows.  Blocks 0, 1
            // are the diagonal of A^{-1} = R(0:32, 0:32)^{-1} (in Ai), blocks 2, 3 that
            // of C^{-1} = R(32:64, 32:64)^{-1} (in Ci); above them A^{-1} and C^{-1} are zero.
            const int g = lane >> 4, j = lane & 15, rb = 16 * g;
            double x[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                double p[4] = {(i == j) ? 1.0 : 0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int k = 0; k < i; ++k) p[k & 3] = fma(-S[(rb + i) * LDS_LD + rb + k], x[k], p[k & 3]);
                const double sacc = (p[0] + p[1]) + (p[2] + p[3]);
                x[i] = (rb + i < jb) ? sacc * invd[rb + i] : ((i == j) ? 1.0 : 0.0);
            }
            double *Xo = (g < 2) ? Ai : Ci;
            const int o = 16 * (g & 1);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                Xo[(o + i) * 33 + o + j] = x[i];
                if (o == 0) Xo[i * 33 + 16 + j] = 0.0;
            }
        }
        __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();
    if (diag) {
        // R_ss goes to B one launch later: the other workgroups of this launch still
        // read the diagonal tile.  It waits in Rscr[s & 1]; R_{s-1,s-1} moves to B now.
        double *Rs = Rscr + (s & 1) * NB * NB;
        for (int idx = tid; idx < NB * NB; idx += blockDim.x) Rs[idx] = S[(idx % NB) * LDS_LD + idx / NB];
        if (s >= 1) put_diag(B, ldb, rows, m, s - 1, Rscr);
        return;
    }
    // the lower-left 16 x 16 blocks of A^{-1} and C^{-1}: -D1^{-1} (R10 D0^{-1}) by wave 0
    // and -D3^{-1} (R32 D2^{-1}) by wave 1, through Eb
    if (wv < 2) {
        const int l = tid & 63, li = l & 15, lk = l >> 4;
        double *Xb = wv ? Ci : Ai;
        const int r0 = wv ? 32 : 0;   // row / column offset of the 32 x 32 block in R_ss
        d4 e = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int k = 4 * ks + lk;
            e = __builtin_amdgcn_mfma_f64_16x16x4f64(S[(r0 + 16 + li) * LDS_LD + r0 + k], Xb[k * 33 + li], e, 0, 0,
                                                     0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) Eb[(16 * wv + 4 * r + lk) * 33 + li] = e[r];
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        d4 f = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int k = 4 * ks + lk;
            f = __builtin_amdgcn_mfma_f64_16x16x4f64(Xb[(16 + li) * 33 + 16 + k], Eb[(16 * wv + k) * 33 + li], f, 0,
                                                     0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) Xb[(16 + 4 * r + lk) * 33 + li] = -f[r];
    }
    __syncthreads();
    // R^{-1}(32:64, 0:32) = F = -C^{-1} (R(32:64, 0:32) A^{-1}): two 32 x 32 x 32 products
    // on the MFMA, wave w forming the 16 x 16 output block (w / 2, w % 2); F replaces
    // the intermediate in Eb, the panel tile replaces R_ss in S
    {
        const int l = tid & 63, li = l & 15, lk = l >> 4;
        const int bi = wv >> 1, bj = wv & 1;
        const bool rowok = 32 + 16 * bi + li < jb;
        d4 e = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            const int k = 4 * ks + lk;
            const double xa = rowok ? S[(32 + 16 * bi + li) * LDS_LD + k] : 0.0;
            const double za = Ai[k * 33 + 16 * bj + li];
            e = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, za, e, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) Eb[(16 * bi + 4 * r + lk) * 33 + 16 * bj + li] = e[r];
        __syncthreads();
        if (wv >= 1) {   // S is free again: the parked panel tile into S
            double co[2][2][4];
            own_rw(t, co, false);
            to_lds(t, co);
            if (wv == 1) {
                const TileIdx t0(0);
                own_rw(t0, co, false);
                to_lds(t0, co);
            }
        }
        d4 f = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            const int k = 4 * ks + lk;
            const double xa = Ci[(16 * bi + li) * 33 + k];
            const double za = Eb[k * 33 + 16 * bj + li];
            f = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, za, f, 0, 0, 0);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) Eb[(16 * bi + 4 * r + lk) * 33 + 16 * bj + li] = -f[r];
    }
    __syncthreads();
    // X = C R_ss^{-T}: R^{-1}(col, k) is A^{-1} (col, k < 32), zero (col < 32 <= k),
    // F (col >= 32, k < 32) or C^{-1} (col, k >= 32); columns < 32 need k < 32 only
    d4 acc[2][2];
    zero_acc(acc);
    {
        const int nks = (t.qc == 0) ? 8 : 16;   // uniform per wave
        double a[2][16], b[2][16];
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            const int k = 4 * ks + t.lk;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int col = 16 * u + t.li;   // within the wave's 32 columns
                a[u][ks] = S[(t.qr + 16 * u + t.li) * LDS_LD + k];
                double rv;
                if (t.qc == 0) rv = (k < 32) ? Ai[col * 33 + k] : 0.0;
                else rv = (k < 32) ? Eb[col * 33 + k] : Ci[col * 33 + (k - 32)];
                b[u][ks] = rv;
            }
        }
#pragma unroll
        for (int ks = 0; ks < 16; ++ks)
            if (ks < nks) {
#pragma unroll
                for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                    for (int tj = 0; tj < 2; ++tj)
                        acc[ti][tj] =
                            __builtin_amdgcn_mfma_f64_16x16x4f64(b[tj][ks], a[ti][ks], acc[ti][tj], 0, 0, 0);
            }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = I0 + t.row(a), k = t.col(b, r);
                if (gi < rows && k < jb) B[gi + ldb * (J0 + k)] = acc[a][b][r];
            }
}

// R^T x = u, R lower (the factor left in B), u read with a stride (row m of B).
// Workgroup q handles block J = T-1-q: it accumulates R(K, J)^T x_K for K > J as
// the blocks x_K are released, then solves with R_JJ^T by backward substitution
// (one wave, lane = row) and releases x_J.
__global__ void __launch_bounds__(256)
k_trsv_bwd_chain(const double *__restrict__ R, int64_t ldb, int m, const double *__restrict__ u, int64_t ustride,
                 double *__restrict__ x, int *__restrict__ flags, int epoch, int *__restrict__ fail) {
    __shared__ double D[NB * LDS_LD];   // R_JJ, row-major
    __shared__ double part[4][NB];
    __shared__ double xk[NB];
    __shared__ int go;
    const int tid = threadIdx.x;
    const int T = (m + NB - 1) / NB;
    const int J = T - 1 - int(blockIdx.x);
    const int J0 = NB * J;
    const int jb = (m - J0 < NB) ? (m - J0) : NB;
    for (int idx = tid; idx < NB * NB; idx += blockDim.x) {
        const int i = idx % NB, j = idx / NB;   // consecutive threads: consecutive rows of column j
        D[i * LDS_LD + j] = (i < jb && j <= i) ? R[(J0 + i) + ldb * (J0 + j)] : 0.0;
    }
    __syncthreads();
    // wave 0, while the later blocks of x are still being formed: lane j holds column j
    // of R_JJ^{-1} (forward substitution, four partial sums per row; identity rows
    // beyond jb), so that x_J = R_JJ^{-T} v becomes one product once v is known
    double rinv[NB];
    if (tid < NB) {
        xk[tid] = (tid < jb) ? 1.0 / D[tid * LDS_LD + tid] : 1.0;
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            double p4[4] = {(i == tid) ? 1.0 : 0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < i; ++k) p4[k & 3] = fma(-D[i * LDS_LD + k], rinv[k], p4[k & 3]);
            const double sacc = (p4[0] + p4[1]) + (p4[2] + p4[3]);
            rinv[i] = (i < jb) ? sacc * xk[i] : ((i == tid) ? 1.0 : 0.0);
        }
    }
    __syncthreads();
    const int jj = tid % NB, pg = tid / NB;   // column jj of the block, rows pg*16 .. pg*16+15 of tile K
    double acc = 0.0;
    for (int K = T - 1; K > J; --K) {
        const int K0 = NB * K;
        const int kb = (m - K0 < NB) ? (m - K0) : NB;
        double rv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int r = pg * 16 + i;
            rv[i] = (r < kb && jj < jb) ? R[(K0 + r) + ldb * (J0 + jj)] : 0.0;
        }
        if (tid == 0) {
            const bool ok = flag_wait(&flags[K], epoch);
            if (!ok) atomicCAS(fail, 0, -1);
            go = ok;
        }
        __syncthreads();
        if (!go) return;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (tid < NB) xk[tid] = (tid < kb) ? x[K0 + tid] : 0.0;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i) acc = fma(rv[i], xk[pg * 16 + i], acc);
        __syncthreads();
    }
    part[pg][jj] = acc;
    __syncthreads();
    if (tid < 64) {
        const int lane = tid;
        double v = (lane < jb) ? u[(J0 + lane) * ustride] : 0.0;
        v -= part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane];
        // x_J(i) = sum_k R_JJ^{-1}(k, i) v_k, v broadcast through LDS
        xk[lane] = v;
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        double p4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < NB; ++k) p4[k & 3] = fma(rinv[k], xk[k], p4[k & 3]);
        v = (p4[0] + p4[1]) + (p4[2] + p4[3]);
        if (lane < jb) x[J0 + lane] = v;
        __threadfence();
        if (lane == 0) flag_release(&flags[J], epoch);
    }
}

__global__ void k_scatter_strided(int m, const double *__restrict__ a, double *__restrict__ b, int64_t stride) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) b[i * stride] = a[i];
}

}  // namespace

int potrf_flag_count(int m) { return (m + NB - 1) / NB + 1; }

size_t potrf_work_doubles(int /*m*/) { return size_t(2) * NB * NB; }

void launch_potrf_rows(int m, int rows, double *B, int64_t ldb, double *work, int *fail, hipStream_t st) {
    const int T_rows = (rows + NB - 1) / NB, T_cols = (m + NB - 1) / NB;
    for (int s = 0; s < T_cols; ++s) {
        const int nt = T_rows - s;
        int nbulk = 0;
        if (s >= 1)
            for (int K = s + 1; K < T_cols; ++K) nbulk += T_rows - K;
        hipLaunchKernelGGL(k_chol_step, dim3(nt + nbulk), dim3(256), 0, st, B, ldb, m, rows, s, fail, work);
    }
    if (T_cols > 0)
        hipLaunchKernelGGL(k_put_diag, dim3(1), dim3(256), 0, st, B, ldb, rows, m, T_cols - 1, (const double *)work);
}

void launch_potrf(int m, double *B, int64_t ldb, double *work, int *fail, hipStream_t st) {
    launch_potrf_rows(m, m, B, ldb, work, fail, st);
}

void launch_potrs_bwd(int m, const double *R, int64_t ldb, const double *u, int64_t ustride, double *x, int *flags,
                      int epoch, int *fail, hipStream_t st) {
    const int T = (m + NB - 1) / NB;
    if (T > 0)
        hipLaunchKernelGGL(k_trsv_bwd_chain, dim3(T), dim3(256), 0, st, R, ldb, m, u, ustride, x, flags, epoch, fail);
}

void launch_set_row(int m, const double *g, double *row, int64_t stride, hipStream_t st) {
    hipLaunchKernelGGL(k_scatter_strided, dim3((m + 255) / 256), dim3(256), 0, st, m, g, row, stride);
}

}  // namespace sdpc
