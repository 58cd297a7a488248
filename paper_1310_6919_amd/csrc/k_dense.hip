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
#include <algorithm>

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

// The same product with the k range loaded in two halves of 32 (half the operand
// registers in flight; kk = 64).
__device__ inline void tile_mma_halves(const TileIdx &t, const double *A, int64_t lda, int ar0, int amax, int ac0,
                                       const double *Bm, int64_t ldbm, int br0, int bmax, int bc0, d4 acc[2][2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        double a[2][8], b[2][8];
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            const int k = 32 * h + 4 * ks + t.lk;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int ra = ar0 + t.qr + 16 * u + t.li, rb = br0 + t.qc + 16 * u + t.li;
                a[u][ks] = (ra < amax) ? A[ra + lda * (ac0 + k)] : 0.0;
                b[u][ks] = (rb < bmax) ? Bm[rb + ldbm * (bc0 + k)] : 0.0;
            }
        }
#pragma unroll
        for (int ks = 0; ks < 8; ++ks)
#pragma unroll
            for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                for (int tj = 0; tj < 2; ++tj)
                    acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[tj][ks], a[ti][ks], acc[ti][tj], 0, 0, 0);
    }
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

// In-LDS factorisation D = R R^T of a 64 x 64 diagonal tile with the 64 rows of a
// second tile C riding along, which leaves X = C R^{-T} in them (the panel solve of
// the column comes with the factorisation).  Four panels of 16 columns:
//   elimination  every participating wave holds the 16 pivot rows in lanes 0..15
//                and up to 48 further rows (D rows below the panel, then C rows) in
//                lanes 16..63, and eliminates the panel in registers (elim_lds);
//                wave 0 writes the pivot rows back, every lane its other row;
//   update       the rows below the panel and the C rows lose the rank-16 product
//                of their panel columns with those of the D rows, 16 x 16 blocks on
//                the MFMA straight from LDS (blocks above D's diagonal skipped).
// D is read as it stands, without masks:
//   * entries above the diagonal of a pivot row are replaced by 0 at their own step
//     before anything reads them (a lane above the pivot gets a zero multiplier);
//   * columns at or beyond jb (padding of the last block, with their pivots) feed
//     only columns at or beyond jb, since the elimination only moves values to the
//     right, and those are neither stored nor checked: padded pivots may be anything;
//   * a row at or beyond jb that exists (a right-hand-side row riding along the last
//     block) is eliminated like any other row in the first jb columns, whether it
//     sits among the pivot rows or below them.
// S and Cs are row-major with row length LDS_LD.  On return S holds R in its first
// jb columns on and below the diagonal (other entries unspecified) and Cs holds X in
// its first jb columns.  With check, a pivot among the first jb that was not
// positive and finite sets fail = J0 + its 1-based index (the first report wins).
__device__ inline void factor64_ride(double *S, double *Cs, bool has_c, int jb, double (*Wl)[64], bool check,
                                     int *fail, int J0) {
    const int wv = int(threadIdx.x) >> 6, lane = int(threadIdx.x) & 63;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll 1
    for (int c0 = 0; c0 < NB; c0 += 16) {
        const int nD = NB - 16 - c0;              // D rows below the panel's pivot rows
        const int nR = nD + (has_c ? NB : 0);     // rows riding along the panel
        const int q = 48 * wv + lane - 16;        // riding row of lanes 16..63
        if (wv == 0 || 48 * wv < nR) {            // uniform
            __builtin_amdgcn_s_setprio(3);        // the chain: ahead of co-resident bulk work
            // the lane's row: a D row (a pivot or one below the panel), a C row, or none
            // (then a pivot row is read and nothing is stored)
            const bool pivot = lane < 16, dro = pivot || q < nD, cro = !dro && q < nR;
            const int r = pivot ? c0 + lane : (dro ? c0 + 16 + q : (cro ? q - nD : c0 + li));
            double *row = ((dro || !cro) ? S : Cs) + r * LDS_LD + c0;
            double a[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) a[t] = row[t];
            elim_lds<16>(a, 0, Wl[wv]);
            if ((pivot && wv == 0) || (!pivot && (dro || cro))) {
#pragma unroll
                for (int t = 0; t < 16; ++t) row[t] = a[t];
            }
            if (check && wv == 0) {
                double dg = 0.0;
#pragma unroll
                for (int t = 0; t < 16; ++t)
                    if (t == lane) dg = a[t];
                const unsigned long long bad = __ballot(pivot && r < jb && !((dg > 0.0) && isfinite(dg)));
                if (bad != 0ull && lane == 0) atomicCAS(fail, 0, J0 + c0 + __ffsll((long long)bad));
            }
            __builtin_amdgcn_s_setprio(0);
        }
        __syncthreads();
        if (nD == 0) break;   // uniform: the last panel has no trailing columns
        // trailing update: output blocks of 16 x 16, rows of D below the panel (row block
        // rb >= column block cb) or of C (row block rc), columns c0 + 16 + 16 cb; block bi
        // of the list goes to wave bi % 4
        const int nb = nD / 16;
        const int nDb = nb * (nb + 1) / 2;
        const int nblk = nDb + (has_c ? 4 * nb : 0);
        for (int bi = wv; bi < nblk; bi += 4) {
            int rb = 0, cb = 0;
            double *O;
            if (bi < nDb) {
                int t = bi;
                while (t > rb) {
                    t -= rb + 1;
                    ++rb;
                }
                cb = t;
                O = S + (c0 + 16 + 16 * rb) * LDS_LD;
            } else {
                rb = (bi - nDb) / nb;
                cb = (bi - nDb) % nb;
                O = Cs + 16 * rb * LDS_LD;
            }
            const double *Z = S + (c0 + 16 + 16 * cb) * LDS_LD;
            d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(O[li * LDS_LD + c0 + 4 * ks + lk],
                                                           Z[li * LDS_LD + c0 + 4 * ks + lk], acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) O[(4 * r + lk) * LDS_LD + c0 + 16 + 16 * cb + li] -= acc[r];
        }
        __syncthreads();
    }
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
    const int tid = threadIdx.x, wv = tid >> 6;
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
    // (factor64_ride), which leaves X = C R_ss^{-T} in them: the factorisation is the
    // whole solve.
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
    factor64_ride(S, Cs, !diag, jb, Wl, diag, fail, J0);
    if (!diag) {
        for (int idx = tid; idx < NB * NB; idx += blockDim.x) {   // X = C R_ss^{-T}
            const int r = idx % NB, k = idx / NB;
            if (I0 + r < rows && k < jb) B[(I0 + r) + ldb * (J0 + k)] = Cs[r * LDS_LD + k];
        }
    } else {
        // R_ss parks column-major in Rscr[s & 1] (this launch's column workgroups read
        // D_ss from B); R_{s-1,s-1} moves from Rscr[(s - 1) & 1] to B
        for (int idx = tid; idx < NB * NB; idx += blockDim.x) {
            const int i = idx % NB, k = idx / NB;
            Rs[idx] = (k <= i) ? S[i * LDS_LD + k] : 0.0;
        }
        if (s >= 1) {
            const int Jp = J0 - NB;   // block s-1 is a full 64-wide block
            const double *Rp = Rscr + ((s - 1) & 1) * NB * NB;
            for (int idx = tid; idx < NB * NB; idx += blockDim.x) {
                const int i = idx % NB, k = idx / NB;
                if (Jp + i < rows && k <= i) B[(Jp + i) + ldb * (Jp + k)] = Rp[idx];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Dataflow form, one launch per factorisation, column-synchronous like the column
// steps above but without their launch boundaries.  Two kinds of task:
//   updater s       D_s minus the panels 0 .. s-2 (left-looking, in MFMA
//                   accumulators), parked column-major in the workspace Dp[s];
//   column task     one per tile (I, s), I > s (or one with no tile when the column
//                   has none below the diagonal): the tile minus the panels 0 .. s-1,
//                   then D_s from Dp[s] minus panel s-1, factorised with the tile's
//                   rows riding along (factor64_ride), which leaves X(I, s) in them.
//                   The first task of the column also stores R_s and checks the pivots.
// Every tile of column s is finished one factorisation after panel s-1 arrives, so
// no triangular solve waits on the chain of diagonal factors.  The tasks' own SCM
// values depend on no other task and are fetched while the first panels are awaited.
// Task order: U0, U1, C0, U2, C1, ..., U_{T-1}, C_{T-2}, C_{T-1} (Cs: the column
// tasks of column s), so every dependency of a task has a lower workgroup index and
// was dispatched before it (each XCD dispatches its workgroups in order), and the
// waits, bounded spins on flags holding the call's epoch, cannot deadlock: the
// lowest unfinished task always holds a slot and has its inputs.  A wait that runs
// out sets fail = -1, after which no task waits any more (every task still runs to
// its end and releases its flag).
struct FlowTask {
    int s, I;   // column; tile row of a column task (-1: none)
    bool upd;
};

__device__ __host__ inline FlowTask flow_task(int id, int T_rows, int T_cols) {
    if (id == 0) return {0, -1, true};
    --id;
    for (int s = 0; s < T_cols; ++s) {
        if (s + 1 < T_cols) {
            if (id == 0) return {s + 1, -1, true};
            --id;
        }
        const int nc = T_rows - s - 1, n = nc > 0 ? nc : 1;
        if (id < n) return {s, nc > 0 ? s + 1 + id : -1, false};
        id -= n;
    }
    return {-1, -1, false};
}

// Polls are relaxed loads: an acquire load at agent scope invalidates the
// caches on every poll, and hundreds of resident waiting workgroups doing that
// keep every XCD's L2 cold.  The caller issues one acquire fence after the
// flags it needs have been seen.
__device__ inline bool flow_poll(const int *flag, int epoch, int *fail) {
    for (int it = 0; it < kSpinLimit; ++it) {
        if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch) return true;
        if (__hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < 0) return false;
        __builtin_amdgcn_s_sleep(2);
    }
    atomicCAS(fail, 0, -1);
    return false;
}

__device__ inline bool flow_is_set(const int *flag, int epoch) {
    return __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch;
}

__global__ void __launch_bounds__(256)
k_chol_flow(double *__restrict__ B, int64_t ldb, int m, int rows, int T_rows, int T_cols, int *__restrict__ ready,
            double *__restrict__ dpart, int epoch, int *__restrict__ fail) {
    __shared__ double S[NB * LDS_LD];
    __shared__ double Cs[NB * LDS_LD];
    __shared__ __attribute__((aligned(16))) double Wl[3][64];
    __shared__ int upto[2];
    const int tid = threadIdx.x, wv = tid >> 6;
    const FlowTask tk = flow_task(int(blockIdx.x), T_rows, T_cols);
    if (tk.s < 0) return;
    const int s = tk.s, K0 = NB * s;
    const int jb = (m - K0 < NB) ? (m - K0) : NB;
    auto flag = [&](int I, int Kc) { return ready + int64_t(I) * T_cols + Kc; };
    int *dflag = ready + int64_t(T_rows) * T_cols + s;   // D_s parked in Dp
    double *Dp = dpart + size_t(s) * NB * NB;
    // Panels p0 .. e-1 (e <= pend) of the tile rows Ia and Ib (Ib < 0: none) ready:
    // thread 0 waits for panel p0, takes every later panel already released, and
    // acquires once for all of them; the barrier hands the acquisition to the other
    // waves.  upto[] alternates so that a fast thread 0 cannot overwrite the value a
    // slow wave has still to read.
    int gathers = 0;
    auto gather = [&](int p0, int pend, int Ia, int Ib) -> int {
        const int slot = (gathers++) & 1;
        if (tid == 0) {
            int e = pend;   // after an abort nothing is waited for any more
            if (flow_poll(flag(Ia, p0), epoch, fail) && (Ib < 0 || flow_poll(flag(Ib, p0), epoch, fail))) {
                e = p0 + 1;
                while (e < pend && flow_is_set(flag(Ia, e), epoch) && (Ib < 0 || flow_is_set(flag(Ib, e), epoch))) ++e;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            upto[slot] = e;
        }
        __syncthreads();
        return upto[slot];
    };
    // the workgroup's stores are ordered before thread 0's release by the barrier
    // (the waves share one vector L1), then one release fence
    auto release = [&](int *f) {
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(f, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    };
    // accumulator quadrants: D by waves 0, 1, 2 (q0, q1, q3; q2 lies above the
    // diagonal), C by waves 0..3 (q3, q2, q0, q1)
    const TileIdx tqd(wv == 2 ? 3 : wv);
    const TileIdx tqc(wv == 0 ? 3 : (wv == 1 ? 2 : wv - 2));
    auto sub_d = [&](const d4 (&acc)[2][2]) {
        if (wv < 3) {
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int gi = K0 + tqd.row(a), lk = tqd.col(b, r);
                        if (gi < rows && lk < jb && gi >= K0 + lk) S[tqd.row(a) * LDS_LD + lk] -= acc[a][b][r];
                    }
        }
    };
    if (tk.upd) {
        // ---- updater s: D_s (lower, zero elsewhere) minus panels 0 .. s-2 into Dp[s]
        for (int idx = tid; idx < NB * NB; idx += blockDim.x) {
            const int r = idx % NB, k = idx / NB;
            S[r * LDS_LD + k] = (K0 + r < rows && k < jb && k <= r) ? B[(K0 + r) + ldb * (K0 + k)] : 0.0;
        }
        d4 accd[2][2];
        zero_acc(accd);
        for (int p = 0; p < s - 1;) {
            const int e = gather(p, s - 1, s, -1);
            for (; p < e; ++p)
                if (wv < 3) tile_mma_halves(tqd, B, ldb, K0, rows, NB * p, B, ldb, K0, m, NB * p, accd);
        }
        __syncthreads();   // the fetch is complete (s <= 1 has no gather)
        sub_d(accd);
        __syncthreads();
        for (int idx = tid; idx < NB * NB; idx += blockDim.x) {
            const int r = idx % NB, k = idx / NB;
            Dp[idx] = S[r * LDS_LD + k];
        }
        release(dflag);
        return;
    }
    // ---- column task: the tile C = (I, s) if any, and the factor of D_s
    const bool has_c = tk.I >= 0;
    const bool first = !has_c || tk.I == s + 1;
    const int I0 = NB * tk.I;
    if (has_c)
        for (int idx = tid; idx < NB * NB; idx += blockDim.x) {
            const int r = idx % NB, k = idx / NB;
            Cs[r * LDS_LD + k] = (I0 + r < rows && k < jb) ? B[(I0 + r) + ldb * (K0 + k)] : 0.0;
        }
    d4 accd[2][2], accc[2][2];
    zero_acc(accd);
    zero_acc(accc);
    // panels 0 .. s-2 of the tile; then D_s from Dp[s] (its updater needs the same
    // panels, so it is usually ready) while panel s-1, the one on the critical path,
    // is still awaited
    if (has_c)
        for (int p = 0; p < s - 1;) {
            const int e = gather(p, s - 1, tk.I, s);
            for (; p < e; ++p) tile_mma_halves(tqc, B, ldb, I0, rows, NB * p, B, ldb, K0, m, NB * p, accc);
        }
    if (tid == 0) {
        flow_poll(dflag, epoch, fail);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    for (int idx = tid; idx < NB * NB; idx += blockDim.x) {
        const int r = idx % NB, k = idx / NB;
        S[r * LDS_LD + k] = Dp[idx];
    }
    if (s >= 1) {
        gather(s - 1, s, has_c ? tk.I : s, has_c ? s : -1);
        if (has_c) tile_mma_halves(tqc, B, ldb, I0, rows, NB * (s - 1), B, ldb, K0, m, NB * (s - 1), accc);
        if (wv < 3) tile_mma_halves(tqd, B, ldb, K0, rows, NB * (s - 1), B, ldb, K0, m, NB * (s - 1), accd);
    }
    __syncthreads();   // D_s is in S
    sub_d(accd);
    if (has_c) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gi = I0 + tqc.row(a), lk = tqc.col(b, r);
                    if (gi < rows && lk < jb) Cs[tqc.row(a) * LDS_LD + lk] -= accc[a][b][r];
                }
    }
    __syncthreads();
    factor64_ride(S, Cs, has_c, jb, Wl, first, fail, K0);
    for (int idx = tid; idx < NB * NB; idx += blockDim.x) {   // X(I, s), and R_s by the first task
        const int r = idx % NB, k = idx / NB;
        if (has_c && I0 + r < rows && k < jb) B[(I0 + r) + ldb * (K0 + k)] = Cs[r * LDS_LD + k];
        if (first && K0 + r < rows && k < jb && k <= r) B[(K0 + r) + ldb * (K0 + k)] = S[r * LDS_LD + k];
    }
    if (has_c) release(flag(tk.I, s));
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

int potrf_flow_flag_count(int m, int rows) {
    const int T_rows = (rows + NB - 1) / NB, T_cols = (m + NB - 1) / NB;
    return T_rows * T_cols + T_cols;
}

size_t potrf_flow_work_doubles(int m) { return size_t((m + NB - 1) / NB) * NB * NB; }

void launch_potrf_flow(int m, int rows, double *B, int64_t ldb, int *flags, double *work, int epoch, int *fail,
                       hipStream_t st) {
    const int T_rows = (rows + NB - 1) / NB, T_cols = (m + NB - 1) / NB;
    if (T_cols <= 0) return;
    int ntask = T_cols;   // updaters
    for (int s = 0; s < T_cols; ++s) ntask += std::max(T_rows - s - 1, 1);
    hipLaunchKernelGGL(k_chol_flow, dim3(ntask), dim3(256), 0, st, B, ldb, m, rows, T_rows, T_cols, flags, work,
                       epoch, fail);
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
