// Dense FP64 Cholesky of the Schur complement matrix, B = R R^T (type (i) of
// Section 3.1), and the backward substitution of the SCE (eq. SCE).
//
// Right-looking, 64-wide column blocks, one fused launch per block column s:
//   workgroups 0..nt-1   tile rows s .. of column block s.  Each applies the
//                        pending panel s-1 to the diagonal tile D and factorises
//                        it in two 32-column panels, one row per lane (pivot row
//                        values broadcast by readlane and through LDS), the update
//                        between the panels on the MFMA.  Workgroup 0 stores R_ss
//                        and reports a failed pivot; every other one also applies
//                        panel s-1 to its own tile C, whose rows ride along the
//                        eliminations (32 per wave) and come out as X = C R_ss^{-T}.
//                        Repeating the small factorisation in every workgroup of
//                        the column spares a hand-over through memory on the
//                        critical path.
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
    __shared__ double S[NB * LDS_LD];    // the updated diagonal tile, row-major; then R(:, 0:32)
    __shared__ double Cs[NB * LDS_LD];   // the updated panel tile, row-major; then X(:, 0:32)
    __shared__ __attribute__((aligned(16))) double Wl[3][64];   // multiplier broadcasts, one row per wave
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
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
    // diagonal tile D = R_ss R_ss^T itself, so no workgroup waits on another; the
    // diagonal workgroup alone reports a failed pivot and stores R_ss.  In the others
    // the 64 rows of the panel tile C ride along the elimination of D as extra rows
    // (32 per wave), which leaves X = C R_ss^{-T} in them: the two 32-column panels
    // of the factorisation are the whole solve.
    const int I = s + int(blockIdx.x), I0 = NB * I;
    const bool diag = (I == s);
    double *Rs = Rscr + (s & 1) * NB * NB;   // R_ss, column-major, until the next launch
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
    auto to_lds = [&](const TileIdx &tq, const double (&c)[2][2][4], double *T) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) T[tq.row(a) * LDS_LD + tq.col(b, r)] = c[a][b][r];
    };
    // quadrant q covers rows 32 (q % 2), columns 32 (q / 2).  D: q0, q1, q3 by waves
    // 0, 1, 2 (q2 lies above the diagonal); C: q3, q2, q0, q1 by waves 0..3
    if (wv < 3) {
        double c[2][2][4];
        const TileIdx tq(wv == 2 ? 3 : wv);
        stage(tq, J0, true, c);
        to_lds(tq, c, S);
    }
    if (!diag) {
        double c[2][2][4];
        const TileIdx tq(wv == 0 ? 3 : (wv == 1 ? 2 : wv - 2));
        stage(tq, I0, false, c);
        to_lds(tq, c, Cs);
    }
    __syncthreads();
    // D as the elimination sees it: rows at or beyond jb, or beyond the matrix, are
    // identity rows in the columns at and beyond jb; rows below jb that exist keep
    // their values in the first jb columns (right-hand-side rows riding along the
    // last block get their forward substitution)
    auto dsel = [&](int i, int k, double v) -> double {
        return (J0 + i < rows && k < jb) ? (k <= i ? v : 0.0) : (i == k ? 1.0 : 0.0);
    };
    // every pivot of the block must have been positive and finite (a failed one
    // leaves a NaN on the diagonal); lanes 0..31 of wave w hold pivots r0 + lane
    auto check_pivots = [&](const double (&a)[32], int r0) {
        double dg = 0.0;
#pragma unroll
        for (int k = 0; k < 32; ++k)
            if (k == lane) dg = a[k];
        const unsigned long long badm = __ballot(lane < 32 && r0 + lane < jb && !((dg > 0.0) && isfinite(dg)));
        if (badm != 0ull && lane == 0) atomicCAS(fail, 0, J0 + r0 + __ffsll((long long)badm));
    };
    // panel 1 (columns 0..31): lanes 0..31 hold the pivot rows D(0:32, :); lanes
    // 32..63 ride along with D(32:64, :) (wave 2) or C rows 32 w .. (waves 0, 1)
    if (wv == 2 || (!diag && wv < 2)) {
        __builtin_amdgcn_s_setprio(3);   // the chain of the launch: ahead of the bulk waves on this CU
        const bool crow = wv < 2 && lane >= 32;
        const int ci = 32 * wv + lane - 32;   // C row of a riding lane
        const double *src = crow ? Cs + ci * LDS_LD : S + lane * LDS_LD;
        double a[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            const double v = src[k];
            a[k] = crow ? v : dsel(lane, k, v);
        }
        elim32_lds(a, 0, Wl[wv]);
        if (crow) {
#pragma unroll
            for (int k = 0; k < 32; ++k) Cs[ci * LDS_LD + k] = a[k];   // X(:, 0:32)
        } else if (wv == 2) {
#pragma unroll
            for (int k = 0; k < 32; ++k) S[lane * LDS_LD + k] = a[k];   // R(:, 0:32)
            if (diag) {
                check_pivots(a, 0);
#pragma unroll
                for (int k = 0; k < 32; ++k) Rs[lane + NB * k] = a[k];
            }
        }
        __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();
    // the right halves lose [R(32:64, 0:32); X(:, 0:32)] R(32:64, 0:32)^T: 16 x 16
    // output blocks (rb, cb), rows 16 rb of D(32:64, :) (rb < 2) or of C (rb >= 2),
    // columns 32 + 16 cb; block (0, 1) lies above the diagonal.  Lane l supplies
    // X(l % 16, l / 16) and Z(l / 16, l % 16); result element r: (4 r + l / 16, l % 16).
    {
        const int li = lane & 15, lk = lane >> 4;
        for (int b = wv; b < 12; b += 4) {
            const int rb = b >> 1, cb = b & 1;
            if ((rb == 0 && cb == 1) || (diag && rb >= 2)) continue;   // uniform
            double *O = (rb < 2) ? S + (32 + 16 * rb) * LDS_LD : Cs + 16 * (rb - 2) * LDS_LD;
            const double *Z = S + (32 + 16 * cb) * LDS_LD;
            d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < 8; ++ks)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(O[li * LDS_LD + 4 * ks + lk], Z[li * LDS_LD + 4 * ks + lk],
                                                           acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) O[(4 * r + lk) * LDS_LD + 32 + 16 * cb + li] -= acc[r];
        }
    }
    __syncthreads();
    // panel 2 (columns 32..63): lanes 0..31 hold the pivot rows D(32:64, 32:64); lanes
    // 32..63 ride along with C rows 32 w .. (waves 0, 1) or zeros (diagonal workgroup).
    // Meanwhile waves 2, 3 store X(:, 0:32), or in the diagonal workgroup waves 1..3
    // move R_{s-1,s-1} from Rscr to B.
    if (wv == 0 || (!diag && wv == 1)) {
        __builtin_amdgcn_s_setprio(3);
        const bool crow = lane >= 32;
        const int ci = 32 * wv + lane - 32;
        const double *src = crow ? Cs + (diag ? 0 : ci) * LDS_LD + 32 : S + (32 + lane) * LDS_LD + 32;
        double a[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            const double v = src[k];
            a[k] = crow ? (diag ? 0.0 : v) : dsel(32 + lane, 32 + k, v);
        }
        elim32_lds(a, 0, Wl[wv]);
        if (diag) {
            check_pivots(a, 32);
            if (!crow) {
#pragma unroll
                for (int k = 0; k < 32; ++k) Rs[(32 + lane) + NB * (32 + k)] = a[k];   // R(32:64, 32:64)
            }
        } else if (crow) {
            const int gi = I0 + ci;
#pragma unroll
            for (int k = 0; k < 32; ++k)
                if (gi < rows && 32 + k < jb) B[gi + ldb * (J0 + 32 + k)] = a[k];   // X(:, 32:64)
        }
        __builtin_amdgcn_s_setprio(0);
    } else if (!diag) {
        for (int idx = tid - 128; idx < NB * 32; idx += 128) {
            const int r = idx % NB, k = idx / NB;
            if (I0 + r < rows && k < jb) B[(I0 + r) + ldb * (J0 + k)] = Cs[r * LDS_LD + k];
        }
    } else if (s >= 1) {
        const int Jp = J0 - NB;   // block s-1 is a full 64-wide block
        const double *Rp = Rscr + ((s - 1) & 1) * NB * NB;
        for (int idx = tid - 64; idx < NB * NB; idx += 192) {
            const int i = idx % NB, k = idx / NB;
            if (Jp + i < rows && k <= i) B[(Jp + i) + ldb * (Jp + k)] = Rp[idx];
        }
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
