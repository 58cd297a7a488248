// C ABI of the matrix-completion PDIPM hot path (see include/sdpc.h).
//
// sdpc_create  host symbolic phase (symbolic.cpp) + every index map the
//              kernels need, then one upload; all device workspace is
//              allocated here and nowhere else.
// scm phase    Y = N N^T, Lhat by Algorithm 1, X^ = Lhat^{-T} Lhat^{-1} and
//              Y^{-1} = N^{-T} N^{-1} column by column, B (eq. SCM / newSCM2),
//              optional Cholesky of B.
// sdpc_step    Section 2.2, Steps 1-4: stopping test, HKM direction (SCE,
//              dY, dX on E by eq. newdX2), step lengths (eq. primal_length2
//              clique by clique; the dual one by a parallel positive-
//              definiteness test of Y + alpha dY on many alphas at once),
//              update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <queue>
#include <string>
#include <vector>

#include "../../include/sdpc.h"
#include "kernels.h"
#include "symbolic.h"

using namespace sdpc;

namespace {

// Dual step, one wave per candidate: round 0 tests 511 log-spaced points (neighbours
// 3.7% apart) and the gamma twin of alpha = 1, 512 candidates, two waves per compute
// unit (a candidate's chain runs ~25% faster than with four); round 1 tests 384 even
// points inside the bracket (relative spacing ~9.6e-5) and their 384 gamma twins.
constexpr int kDualRounds = 2;
constexpr int kDualTest[kDualRounds] = {511, 384};
constexpr int kMaxDualRounds = 16;
constexpr int kCand = 1024;      // the most candidates of a round
// the phase flags (8 ints), the scalars (16 doubles) and the dual bracket (4 doubles)
constexpr size_t kReadback = 8 * sizeof(int) + 16 * sizeof(double) + 4 * sizeof(double);
// the next iteration's Schur complement phase is enqueued ahead unless the relative
// gap is already within this factor of the stopping tolerance
constexpr double kAheadGap = 30.0;
constexpr int kMaxClique = 64;   // largest clique of the clique kernels (register tiles of 64 x 64)
constexpr int kMaxPanel = 4096;  // largest storage panel (doubles): 32 KiB of LDS
constexpr int kMaxM = 65535;     // most constraints

struct Timer {
    hipEvent_t a{}, b{};
};

}  // namespace

struct sdpc_handle {
    hipStream_t st = nullptr;
    int n = 0, m = 0;
    sdpc_params prm{};
    Symbolic S;
    SolveSlots slots;    // the multi-right-hand-side substitutions
    SolveSlots wslots;   // the single-product walks (slots freed one block late)
    DevStruct d;
    std::vector<void *> allocs;
    size_t bytes = 0;
    std::string err;
    // host mirrors
    std::vector<int64_t> kq_ptr_h;
    double bmax = 0.0, a0max = 0.0;
    std::vector<int> slot_row_h, slot_col_h;
    // state (E-vectors unless noted)
    double *X = nullptr, *Y = nullptr, *z = nullptr, *G = nullptr;
    double *Xn = nullptr;   // the next X, formed before the iteration is known to have succeeded
    double *dX = nullptr, *dY = nullptr, *dz = nullptr;
    double *N = nullptr, *Lhat = nullptr, *DinvN = nullptr, *DinvL = nullptr;
    double *GN = nullptr, *GL = nullptr;   // walk matrices [D_b^{-1}; P21_b D_b^{-1}] of N and Lhat
    double *Dblk = nullptr;   // factorization 1: D of X^ = L^T D L, w x w per storage block (Lhat holds L^{-1})
    double *Xh = nullptr, *Yi = nullptr, *W = nullptr, *T = nullptr;   // dense n x n, support work
    double *B = nullptr, *g = nullptr, *hcol = nullptr;
    double *scal = nullptr, *alpha_cl = nullptr, *alpha_hi = nullptr, *alphas = nullptr, *cand = nullptr, *part = nullptr;
    double *ccwork = nullptr; // blocks of the column-compressed general SCM (cc_work_doubles)
    double *ubuf = nullptr;   // pending updates of the one-wave factorisations, d.nU per candidate
    double *mwork = nullptr;  // partial results of the metrics
    double *ydw = nullptr, *ydw_dual = nullptr;   // (Y, dY) panel tiles of the Y factor / dual step
    int *flags = nullptr;   // [0..kCand) dual-step candidates, [kCand] dinv, [kCand+1] algorithm 1, [kCand+2]
                            // potrf, [kCand+3] / [kCand+4] algorithm 1 / dinv of the next X, [kCand+5] Y factor
    // flags, scal and alphas are one device block in that order, so that the phase
    // flags, the scalars and the dual bracket are contiguous (kReadback bytes from
    // flags + kCand) and come back in one copy into this pinned host buffer
    unsigned char *rbh = nullptr;
    bool flags_zeroed = false;   // the last operation on flags was the clear enqueued after a step's readback
    bool scm_ready = false;      // the Schur complement phase of the current iterate is already enqueued (by
                                 // the previous step, behind its readback, with N the dual step's twin factor)
    int64_t ldb = 0;
    double last_alpha[2] = {0, 0};
    double scm_ms[5] = {0, 0, 0, 0, 0};
    hipEvent_t ev[8]{};    // phases of an iteration
    hipEvent_t evs[2][6]{};   // phases of the SCM evaluation, two sets used in turn (the next
                              // iteration's may be enqueued before this one's are read)
    int evs_set = 0;          // the set the last SCM evaluation used
    hipEvent_t ev_rb = nullptr;   // a step's readback has landed in rbh
    hipStream_t side = nullptr;   // second stream (default priority): dual step alongside dX and alpha_p
    hipEvent_t ev_dy = nullptr, ev_dual = nullptr;
    int *pflags_b = nullptr;   // hand-over flags of the SCE backward solve
    int *pflags_f = nullptr;   // tile flags of the one-launch SCM Cholesky
    int epoch_f = 0;           // last epoch used on those flags
    double *pwork = nullptr;   // diagonal factors of the SCM Cholesky waiting for the next launch
    double *pwork_f = nullptr; // diagonal blocks parked by the one-launch SCM Cholesky
    int epoch = 0;                                    // last epoch used on those flags
    int next_cand = -1;   // dual-step candidate holding the factor of the current Y, or -1
    bool xside_ready = false;   // Lhat and its diagonal inverses already belong to the current X
    bool metrics_ready = false; // msc holds the metrics of the current iterate (read with the last step)
    double msc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int iters = 0;
    int dual_rounds = 0;            // schedule of the dual step's rounds
    int dual_test[16] = {0};
};

namespace sdpc {

// detail of the last failed call that has no handle (per host thread)
std::string &unbound_error() {
    static thread_local std::string e = "no error";
    return e;
}

void set_unbound_error(const std::string &msg) { unbound_error() = msg; }

}  // namespace sdpc

namespace {

sdpc_status fail(sdpc_handle *h, sdpc_status s, const std::string &msg) {
    if (h) h->err = msg;
    return s;
}

#define HIPCHK(h, call)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail(h, SDPC_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));       \
    } while (0)

template <class Tp>
sdpc_status dalloc(sdpc_handle *h, Tp **p, size_t count) {
    void *q = nullptr;
    const size_t nbytes = std::max<size_t>(count, 1) * sizeof(Tp);
    if (hipMalloc(&q, nbytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, SDPC_E_OOM, "device allocation of " + std::to_string(nbytes) + " bytes failed");
    }
    h->allocs.push_back(q);
    h->bytes += nbytes;
    *p = static_cast<Tp *>(q);
    return SDPC_OK;
}

template <class Tp>
sdpc_status upload(sdpc_handle *h, const Tp **dst, const std::vector<Tp> &src) {
    Tp *p = nullptr;
    sdpc_status s = dalloc(h, &p, src.size());
    if (s != SDPC_OK) return s;
    if (!src.empty()) HIPCHK(h, hipMemcpyAsync(p, src.data(), src.size() * sizeof(Tp), hipMemcpyHostToDevice, h->st));
    *dst = p;
    return SDPC_OK;
}

#define TRY(x)                              \
    do {                                    \
        sdpc_status s_ = (x);               \
        if (s_ != SDPC_OK) return s_;       \
    } while (0)

struct Entry {
    int pi, pj;   // positions, pi >= pj
    double v;
};

}  // namespace

extern "C" {

sdpc_params sdpc_default_params(void) {
    sdpc_params p;
    p.gap_tol = 1e-7;
    p.feas_tol = 1e-7;
    p.beta_feas = 0.1;
    p.beta_infeas = 0.2;
    p.gamma = 0.9;
    p.lambda0 = 100.0;
    p.max_iter = 100;
    p.ordering = 0;
    p.block_width = 32;
    p.verbose = 0;
    p.pool_lds_bytes = 32 * 1024;
    p.solve_kernel = 0;
    p.factorization = 0;
    p.merge_siblings = 1;
    p.dual_points = 0;
    p.chol_kernel = 0;
    p.user_perm = nullptr;
    return p;
}

const char *sdpc_status_string(sdpc_status s) {
    switch (s) {
        case SDPC_OK: return "ok";
        case SDPC_E_ARG: return "invalid argument";
        case SDPC_E_PATTERN: return "unsupported structure";
        case SDPC_E_NOT_PD: return "matrix not positive definite";
        case SDPC_E_HIP: return "HIP runtime error";
        case SDPC_E_MAXITER: return "iteration limit reached";
        case SDPC_E_STAGNATION: return "stagnation";
        case SDPC_E_NUMERIC: return "non-finite values";
        case SDPC_E_OOM: return "out of device memory";
    }
    return "unknown status";
}

const char *sdpc_last_error(const sdpc_handle *h) { return h ? h->err.c_str() : unbound_error().c_str(); }

void sdpc_destroy(sdpc_handle *h) {
    if (!h) return;
    if (h->st) (void)hipStreamSynchronize(h->st);
    if (h->side) (void)hipStreamSynchronize(h->side);
    for (void *p : h->allocs) (void)hipFree(p);
    for (auto &e : h->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &set : h->evs)
        for (auto &e : set)
            if (e) (void)hipEventDestroy(e);
    if (h->ev_rb) (void)hipEventDestroy(h->ev_rb);
    if (h->ev_dy) (void)hipEventDestroy(h->ev_dy);
    if (h->ev_dual) (void)hipEventDestroy(h->ev_dual);
    if (h->side) (void)hipStreamDestroy(h->side);
    if (h->rbh) (void)hipHostFree(h->rbh);
    delete h;
}

static sdpc_status check_problem(const sdpc_problem *prob, sdpc_handle *h) {
    const int n = prob->n, m = prob->m;
    if (h->prm.block_width < 1 || h->prm.block_width > 32) return fail(h, SDPC_E_ARG, "block_width must be 1..32");
    if (h->prm.pool_lds_bytes < 0 || h->prm.pool_lds_bytes > 64 * 1024)
        return fail(h, SDPC_E_ARG, "pool_lds_bytes must be 0..65536");
    if (h->prm.gamma <= 0 || h->prm.gamma >= 1) return fail(h, SDPC_E_ARG, "gamma must be in (0,1)");
    if (h->prm.solve_kernel < 0 || h->prm.solve_kernel > 1) return fail(h, SDPC_E_ARG, "solve_kernel must be 0 or 1");
    if (h->prm.factorization < 0 || h->prm.factorization > 1)
        return fail(h, SDPC_E_ARG, "factorization must be 0 or 1");
    if (h->prm.chol_kernel < 0 || h->prm.chol_kernel > 1) return fail(h, SDPC_E_ARG, "chol_kernel must be 0 or 1");
    if (h->prm.dual_points != 0 && (h->prm.dual_points < 2 || h->prm.dual_points > 511))
        return fail(h, SDPC_E_ARG, "dual_points must be 0 or 2..511");
    const int64_t nnz = prob->ptr[m + 1];
    if (prob->ptr[0] != 0 || nnz < 0) return fail(h, SDPC_E_ARG, "ptr must start at 0");
    for (int k = 0; k <= m; ++k)
        if (prob->ptr[k + 1] < prob->ptr[k]) return fail(h, SDPC_E_ARG, "ptr not monotone");
    for (int64_t t = 0; t < nnz; ++t) {
        const int r = prob->row[t], c = prob->col[t];
        if (r < 0 || r >= n || c < 0 || c >= n || r < c)
            return fail(h, SDPC_E_ARG, "entry " + std::to_string(t) + " is not a lower-triangle index");
        if (!std::isfinite(prob->val[t])) return fail(h, SDPC_E_ARG, "non-finite value in A");
    }
    for (int k = 0; k < m; ++k)
        if (!std::isfinite(prob->b[k])) return fail(h, SDPC_E_ARG, "non-finite b");
    return SDPC_OK;
}

// lower-triangle aggregate pattern (original indices, diagonal included), then the symbolic phase
static sdpc_status analyze_impl(const sdpc_problem *prob, sdpc_handle *h, std::vector<int> &arow,
                                std::vector<int> &acol) {
    const int n = prob->n, m = prob->m;
    const int64_t nnz = prob->ptr[m + 1];
    {
        std::vector<std::pair<int, int>> e;
        e.reserve(size_t(nnz) + n);
        for (int i = 0; i < n; ++i) e.push_back({i, i});
        for (int64_t t = 0; t < nnz; ++t) e.push_back({prob->row[t], prob->col[t]});
        std::sort(e.begin(), e.end());
        e.erase(std::unique(e.begin(), e.end()), e.end());
        for (auto &p : e) {
            arow.push_back(p.first);
            acol.push_back(p.second);
        }
    }
    SymbolicOptions so;
    so.ordering = h->prm.ordering;
    so.user_perm = h->prm.user_perm;
    so.block_width = h->prm.block_width;
    so.max_block_entries = kMaxPanel;
    so.merge_siblings = h->prm.merge_siblings ? 1 : 0;
    const std::string serr = build_symbolic(n, arow, acol, so, h->S);
    if (!serr.empty()) return fail(h, SDPC_E_PATTERN, serr);
    const Symbolic &S = h->S;
    if (S.max_clique > kMaxClique)
        return fail(h, SDPC_E_PATTERN, "largest clique has " + std::to_string(S.max_clique) + " members (limit " +
                                           std::to_string(kMaxClique) + ")");
    if (S.nslot >= (int64_t(1) << 31)) return fail(h, SDPC_E_PATTERN, "storage exceeds 2^31 entries");
    h->slots = build_solve_slots(S, false);
    h->wslots = build_solve_slots(S, true);
    h->d.n = n;
    h->d.nfwd = h->slots.nfwd;
    h->d.nbwd = h->slots.nbwd;
    h->d.wk_nfwd = h->wslots.nfwd;
    h->d.wk_nbwd = h->wslots.nbwd;
    h->d.max_h = S.max_h;
    h->d.max_w = S.max_w;
    h->d.max_panel = 0;
    for (int b = 0; b < S.nb; ++b)
        h->d.max_panel = std::max<int64_t>(h->d.max_panel, (S.bl_rptr[b + 1] - S.bl_rptr[b]) *
                                                                int64_t(S.bl_first[b + 1] - S.bl_first[b]));
    if (h->prm.factorization == 1)
        for (int r = 0; r < S.ncl; ++r)
            if (S.col_block[S.cl_first[r]] != S.col_block[S.cl_first[r + 1] - 1])
                return fail(h, SDPC_E_PATTERN, "factorization 1 needs every supernode inside one storage block (clique " +
                                                   std::to_string(r) + " has " +
                                                   std::to_string(S.cl_first[r + 1] - S.cl_first[r]) +
                                                   " columns, wider than block_width)");
    if (solve_tile_width(h->d) == 0)
        return fail(h, SDPC_E_PATTERN, "substitution frontier too wide for LDS (" + std::to_string(h->d.nfwd) + "+" +
                                           std::to_string(h->d.nbwd) + " live rows)");
    return SDPC_OK;
}

static sdpc_status create_impl(const sdpc_problem *prob, const sdpc_params *params, hipStream_t stream,
                               sdpc_handle *h) {
    const int n = prob->n, m = prob->m;
    h->st = stream;
    h->n = n;
    h->m = m;
    h->prm = params ? *params : sdpc_default_params();
    TRY(check_problem(prob, h));
    // dual-step schedule: round 0 a log grid of P points over [1e-8, 1], every later
    // round P even points inside the bracket, until the bracket is narrower than 5e-5
    // of its lower end
    if (h->prm.dual_points == 0) {
        h->dual_rounds = kDualRounds;
        for (int r = 0; r < kDualRounds; ++r) h->dual_test[r] = kDualTest[r];
    } else {
        const int P = h->prm.dual_points;
        double width = std::pow(10.0, 8.0 / (P - 1)) - 1.0;
        h->dual_rounds = 1;
        h->dual_test[0] = P;
        while (width > 5e-5 && h->dual_rounds < kMaxDualRounds) {
            h->dual_test[h->dual_rounds++] = P;
            width /= (P + 1);
        }
    }
    std::vector<int> arow, acol;
    TRY(analyze_impl(prob, h, arow, acol));
    const Symbolic &S = h->S;
    DevStruct &d = h->d;
    d.n = n;
    d.m = m;
    d.nb = S.nb;
    d.ncl = S.ncl;
    d.nslot = S.nslot;
    d.max_h = S.max_h;
    d.max_w = S.max_w;
    d.max_clique = S.max_clique;
    if (m > kMaxM) return fail(h, SDPC_E_PATTERN, "more than " + std::to_string(kMaxM) + " constraints");
    d.solve_generic = h->prm.solve_kernel;
    // ---- block arrays
    std::vector<int> fs(S.bl_rows.size()), bs(S.bl_rows.size());
    for (size_t t = 0; t < S.bl_rows.size(); ++t) {
        fs[t] = h->slots.fwd[S.bl_rows[t]];
        bs[t] = h->slots.bwd[S.bl_rows[t]];
    }
    for (int b = 0; b < S.nb; ++b) {
        const int w = S.bl_first[b + 1] - S.bl_first[b];
        for (int64_t t = S.bl_rptr[b] + w; t < S.bl_rptr[b + 1]; ++t)
            if (fs[t] < 0 || bs[t] < 0) return fail(h, SDPC_E_PATTERN, "internal: solve slot missing");
    }
    std::vector<int64_t> dinv_off(S.nb + 1, 0), up_ptr(S.nb + 1, 0);
    std::vector<int> up_pair, up_slot;
    for (int b = 0; b < S.nb; ++b) {
        const int F = S.bl_first[b], w = S.bl_first[b + 1] - F;
        const int64_t r0 = S.bl_rptr[b];
        const int hp = int(S.bl_rptr[b + 1] - r0) - w;
        dinv_off[b + 1] = dinv_off[b] + int64_t(w) * w;
        for (int c = 0; c < hp; ++c)
            for (int a = c; a < hp; ++a) {
                up_pair.push_back(a | (c << 16));
                up_slot.push_back(int(S.slot(S.bl_rows[r0 + w + a], S.bl_rows[r0 + w + c])));
            }
        up_ptr[b + 1] = int64_t(up_pair.size());
    }
    // ---- slots of the pending updates of the one-wave factorisation.  An entry that
    // receives updates is alive from its first update (in block order) until its own
    // block forms its panel; a pool slot freed at a block can be taken by an entry born
    // at the same block (the panel is read before the block's updates are written).
    std::vector<int> up_u(up_slot.size(), -1), slot_u(size_t(S.nslot), -1);
    {
        std::vector<int> born_at(size_t(S.nslot), -1), own(size_t(S.nslot), -1);
        for (int b = 0; b < S.nb; ++b)
            for (int64_t s = S.bl_off[b]; s < S.bl_off[b + 1]; ++s) own[s] = b;
        for (int b = 0; b < S.nb; ++b)
            for (int64_t t = up_ptr[b]; t < up_ptr[b + 1]; ++t)
                if (up_slot[t] >= 0 && born_at[up_slot[t]] < 0) born_at[up_slot[t]] = b;
        std::vector<std::vector<int>> born(S.nb), dies(S.nb);
        int ntarget = 0;
        for (int64_t s = 0; s < S.nslot; ++s)
            if (born_at[s] >= 0) {
                born[born_at[s]].push_back(int(s));
                dies[own[s]].push_back(int(s));
                ++ntarget;
            }
        std::priority_queue<int, std::vector<int>, std::greater<int>> freel;
        int used = 0;
        for (int b = 0; b < S.nb; ++b) {
            for (int s : dies[b]) freel.push(slot_u[s]);
            for (int s : born[b]) {
                int k;
                if (!freel.empty()) { k = freel.top(); freel.pop(); } else { k = used++; }
                slot_u[s] = k;
            }
        }
        // the pool is used when the factorisation's LDS stays within the budget (32 KiB by
        // default: four waves per compute unit); two more slots: one stays zero, one
        // takes the results that update nothing
        d.u_pool = (h->prm.pool_lds_bytes > 0 &&
                    wave_chol_lds_bytes(S.max_h, S.max_w, used + 2) <= size_t(h->prm.pool_lds_bytes)) ? 1 : 0;
        if (!d.u_pool) {   // one slot per target entry, in global memory
            int k = 0;
            for (int64_t s = 0; s < S.nslot; ++s)
                if (born_at[s] >= 0) slot_u[s] = k++;
        }
        d.nU = (d.u_pool ? used : ntarget) + 2;
        std::vector<uint8_t> seen(size_t(S.nslot), 0);
        for (int b = 0; b < S.nb; ++b)
            for (int64_t t = up_ptr[b]; t < up_ptr[b + 1]; ++t) {
                const int s = up_slot[t];
                if (s < 0) continue;
                const bool first = !seen[s];
                seen[s] = 1;
                up_u[t] = (slot_u[s] << 1) | (first ? 1 : 0);
            }
        // padding slots (stored but outside E) start from zero: -2, or -3 - slot when
        // they receive updates (fill inside an amalgamated block)
        for (int64_t s = 0; s < S.nslot; ++s)
            if (!S.isE[s]) slot_u[s] = (slot_u[s] >= 0) ? -3 - slot_u[s] : -2;
    }
    // the slot each panel entry adds (the last, zero, slot where there is no update or
    // outside the panel) per 64 x 32 panel tile, in the one-wave factorisation's read
    // order: per group of four columns, per row, the four slots
    std::vector<int> su_rows;
    if (S.max_h <= 64 && S.max_w <= 32) {
        const int zero = int(d.nU - 2);
        su_rows.assign(size_t(S.nb) * 64 * 32, zero);
        for (int b = 0; b < S.nb; ++b) {
            const int w = S.bl_first[b + 1] - S.bl_first[b];
            const int hh = int(S.bl_rptr[b + 1] - S.bl_rptr[b]);
            for (int i = 0; i < hh; ++i)
                for (int k = 0; k < w; ++k) {
                    const int v = slot_u[S.bl_off[b] + i + int64_t(hh) * k];
                    su_rows[((size_t(b) * 8 + k / 4) * 64 + i) * 4 + k % 4] = v >= 0 ? v : (v <= -3 ? -3 - v : zero);
                }
        }
    } else {
        su_rows.assign(1, -2);
    }
    // the update codes in the MFMA lane order, and the block sizes
    std::vector<int> wc_meta(size_t(S.nb) * 4, 0), wc_up(1, -1);
    if (S.max_h <= 64 && S.max_w <= 32) {
        int hpmax = 0;
        for (int b = 0; b < S.nb; ++b) {
            const int w = S.bl_first[b + 1] - S.bl_first[b];
            const int hh = int(S.bl_rptr[b + 1] - S.bl_rptr[b]);
            hpmax = std::max(hpmax, hh - w);
            wc_meta[size_t(b) * 4] = w;
            wc_meta[size_t(b) * 4 + 1] = hh;
            wc_meta[size_t(b) * 4 + 2] = int(S.bl_off[b]);
        }
        d.wc_rt = hpmax <= 32 ? 2 : 4;
        const int rt = d.wc_rt, mt = rt * (rt + 1) / 2;
        wc_up.assign(size_t(S.nb) * mt * 64 * 4, -1);
        for (int b = 0; b < S.nb; ++b) {
            const int hp = int(S.bl_rptr[b + 1] - S.bl_rptr[b]) - (S.bl_first[b + 1] - S.bl_first[b]);
            // pair (a, c), a >= c: up_ptr[b] + c hp - c (c - 1) / 2 + (a - c)
            const int trash = int(d.nU - 1) << 1;
            auto code = [&](int a, int c) {
                if (a >= hp || c >= hp || a < c) return trash;
                const int u = up_u[size_t(up_ptr[b] + int64_t(c) * hp - int64_t(c) * (c - 1) / 2 + (a - c))];
                return u >= 0 ? u : trash;
            };
            int t = 0;
            for (int ti = 0; ti < rt; ++ti)
                for (int tj = 0; tj <= ti; ++tj, ++t)
                    for (int l = 0; l < 64; ++l)
                        for (int r = 0; r < 4; ++r)
                            wc_up[((size_t(b) * mt + t) * 64 + l) * 4 + r] = code(16 * ti + 4 * r + l / 16, 16 * tj + l % 16);
        }
    }
    // ---- cliques
    std::vector<int64_t> cl_ptr(S.ncl + 1, 0), cl_map_ptr(S.ncl + 1, 0);
    std::vector<int> cl_rows, cl_map;
    for (int r = 0; r < S.ncl; ++r) {
        const int f = S.cl_first[r];
        const int64_t s0 = S.sptr[f], s1 = S.sptr[f + 1];
        const int c = int(s1 - s0);
        for (int64_t t = s0; t < s1; ++t) cl_rows.push_back(S.sidx[t]);
        for (int jj = 0; jj < c; ++jj)
            for (int ii = jj; ii < c; ++ii) {
                const int64_t sl = S.slot(S.sidx[s0 + ii], S.sidx[s0 + jj]);
                if (sl < 0) return fail(h, SDPC_E_PATTERN, "internal: clique entry not stored");
                cl_map.push_back(int(sl));
            }
        cl_ptr[r + 1] = int64_t(cl_rows.size());
        cl_map_ptr[r + 1] = int64_t(cl_map.size());
    }
    // ---- per-slot row/col and weights
    std::vector<int> slot_row(S.nslot, -1), slot_col(S.nslot, -1);
    std::vector<double> wE(S.nslot, 0.0);
    for (int b = 0; b < S.nb; ++b) {
        const int F = S.bl_first[b], w = S.bl_first[b + 1] - F;
        const int64_t r0 = S.bl_rptr[b];
        const int hh = int(S.bl_rptr[b + 1] - r0);
        for (int c = 0; c < w; ++c)
            for (int p = 0; p < hh; ++p) {
                const int64_t s = S.bl_off[b] + p + int64_t(hh) * c;
                if (!S.isE[s]) continue;
                slot_row[s] = S.bl_rows[r0 + p];
                slot_col[s] = F + c;
                wE[s] = (slot_row[s] == slot_col[s]) ? 1.0 : 2.0;
            }
    }
    h->slot_row_h = slot_row;
    h->slot_col_h = slot_col;
    // ---- problem entries in positions
    std::vector<std::vector<Entry>> ent(m + 1);
    for (int k = 0; k <= m; ++k)
        for (int64_t t = prob->ptr[k]; t < prob->ptr[k + 1]; ++t) {
            int a = S.pos[prob->row[t]], c = S.pos[prob->col[t]];
            if (a < c) std::swap(a, c);
            if (prob->val[t] != 0.0) ent[k].push_back({a, c, prob->val[t]});
        }
    h->a0max = 0.0;
    for (auto &e : ent[0]) h->a0max = std::max(h->a0max, std::fabs(e.v));
    h->bmax = 0.0;
    for (int k = 0; k < m; ++k) h->bmax = std::max(h->bmax, std::fabs(prob->b[k]));
    // assembly by slot
    std::vector<int64_t> asm_ptr(S.nslot + 1, 0);
    std::vector<int> asm_k;
    std::vector<double> asm_val;
    {
        std::vector<std::pair<int64_t, std::pair<int, double>>> tmp;
        for (int k = 0; k <= m; ++k)
            for (auto &e : ent[k]) tmp.push_back({S.slot(e.pi, e.pj), {k, e.v}});
        std::stable_sort(tmp.begin(), tmp.end(),
                         [](const auto &x, const auto &y) { return x.first < y.first; });
        for (auto &t : tmp) {
            if (t.first < 0) return fail(h, SDPC_E_PATTERN, "internal: aggregate entry not stored");
            asm_ptr[t.first + 1]++;
            asm_k.push_back(t.second.first);
            asm_val.push_back(t.second.second);
        }
        for (int64_t s = 0; s < S.nslot; ++s) asm_ptr[s + 1] += asm_ptr[s];
    }
    // constraints by k
    std::vector<int64_t> con_ptr(m + 2, 0);
    std::vector<int> con_pi, con_pj, con_slot;
    std::vector<double> con_val;
    for (int k = 0; k <= m; ++k) {
        for (auto &e : ent[k]) {
            con_pi.push_back(e.pi);
            con_pj.push_back(e.pj);
            con_slot.push_back(int(S.slot(e.pi, e.pj)));
            con_val.push_back(e.v * (e.pi == e.pj ? 1.0 : 2.0));
        }
        con_ptr[k + 1] = int64_t(con_pi.size());
    }
    // Hadamard form: every A_k (k >= 1) a single diagonal position
    bool had = m > 0;
    std::vector<int> had_pos(m, 0);
    std::vector<double> had_val(m, 0.0);
    for (int k = 1; k <= m && had; ++k) {
        if (ent[k].empty()) { had = false; break; }
        const int p0 = ent[k][0].pi;
        double v = 0.0;
        for (auto &e : ent[k]) {
            if (e.pi != p0 || e.pj != p0) { had = false; break; }
            v += e.v;
        }
        had_pos[k - 1] = p0;
        had_val[k - 1] = v;
    }
    d.hadamard = had ? 1 : 0;
    // general path: A_q full symmetric CSC over its nonzero columns; union support by rows
    std::vector<int64_t> kq_ptr(m + 1, 0), aq_cptr(1, 0);
    std::vector<int> kq_col, aq_row;
    std::vector<double> aq_val;
    std::map<std::pair<int, int>, int64_t> sup;   // (row, col) -> support index
    for (int q = 1; q <= m; ++q) {
        std::vector<std::pair<std::pair<int, int>, double>> full;   // ((col, row), v)
        for (auto &e : ent[q]) {
            full.push_back({{e.pj, e.pi}, e.v});
            if (e.pi != e.pj) full.push_back({{e.pi, e.pj}, e.v});
        }
        std::sort(full.begin(), full.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
        int lastc = -1;
        for (auto &f : full) {
            const int col = f.first.first, row = f.first.second;
            if (col != lastc) {
                kq_col.push_back(col);
                aq_cptr.push_back(aq_cptr.back());
                lastc = col;
            }
            aq_row.push_back(row);
            aq_val.push_back(f.second);
            aq_cptr.back()++;
            sup.emplace(std::make_pair(row, col), 0);
        }
        kq_ptr[q] = int64_t(kq_col.size());
    }
    std::vector<int64_t> S_rowptr(n + 1, 0);
    std::vector<int> S_col;
    {
        int64_t idx = 0;
        for (auto &kv : sup) {
            kv.second = idx++;
            S_rowptr[kv.first.first + 1]++;
            S_col.push_back(kv.first.second);
        }
        for (int i = 0; i < n; ++i) S_rowptr[i + 1] += S_rowptr[i];
    }
    std::vector<int64_t> am_ptr(m + 1, 0), am_sidx;
    std::vector<double> am_val;
    for (int q = 1; q <= m; ++q) {
        for (auto &e : ent[q]) {
            am_sidx.push_back(sup[{e.pi, e.pj}]);
            am_val.push_back(e.v);
            if (e.pi != e.pj) {
                am_sidx.push_back(sup[{e.pj, e.pi}]);
                am_val.push_back(e.v);
            }
        }
        am_ptr[q] = int64_t(am_sidx.size());
    }
    h->kq_ptr_h = kq_ptr;
    // column-compressed general form: strict triangle with the smaller column union,
    // the diagonal, and the rows of every A_q (full symmetric) for the sparse products
    std::vector<int> ccol, ds_v, seg_q, seg_row, seg_col;
    std::vector<int64_t> seg_ptr(1, 0);
    std::vector<double> ucat, dmat, seg_val;
    std::vector<int> dq_few;
    if (!had && m > 0) {
        std::vector<uint8_t> in_up(n, 0), in_lo(n, 0), in_d(n, 0);
        for (int k = 1; k <= m; ++k)
            for (auto &e : ent[k]) {
                if (e.pi != e.pj) {
                    in_up[e.pi] = 1;   // upper entry (pj, pi) sits in column pi
                    in_lo[e.pj] = 1;   // lower entry (pi, pj) sits in column pj
                } else {
                    in_d[e.pi] = 1;
                }
            }
        int nup = 0, nlo = 0;
        for (int i = 0; i < n; ++i) { nup += in_up[i]; nlo += in_lo[i]; }
        const bool use_up = nup <= nlo;
        std::vector<int> cpos(n, -1), dpos(n, -1);
        for (int i = 0; i < n; ++i)
            if (use_up ? in_up[i] : in_lo[i]) { cpos[i] = int(ccol.size()); ccol.push_back(i); }
        for (int i = 0; i < n; ++i)
            if (in_d[i]) { dpos[i] = int(ds_v.size()); ds_v.push_back(i); }
        const int64_t nc = int64_t(ccol.size()), nds = int64_t(ds_v.size());
        const int64_t ucat_len = int64_t(n) * m * nc;
        const int64_t budget = int64_t(1) << 27;   // doubles per work block (1 GiB)
        if (ucat_len <= budget && nds * m <= budget && int64_t(n) * nc * (m + 1) <= budget) {
            d.cc = 1;
            d.nc = int(nc);
            d.nds = int(nds);
            ucat.assign(size_t(std::max<int64_t>(ucat_len, 1)), 0.0);
            dmat.assign(size_t(std::max<int64_t>(nds * m, 1)), 0.0);
            for (int k = 1; k <= m; ++k) {
                std::vector<std::pair<std::pair<int, int>, double>> full;   // ((row, col), v), both triangles
                for (auto &e : ent[k]) {
                    if (e.pi != e.pj) {
                        const int r = use_up ? e.pj : e.pi, c = use_up ? e.pi : e.pj;
                        ucat[size_t(r) + size_t(n) * (size_t(k - 1) * nc + cpos[c])] += e.v;
                        full.push_back({{e.pi, e.pj}, e.v});
                        full.push_back({{e.pj, e.pi}, e.v});
                    } else {
                        dmat[size_t(dpos[e.pi]) + size_t(nds) * (k - 1)] += e.v;
                        full.push_back({{e.pi, e.pi}, e.v});
                    }
                }
                std::sort(full.begin(), full.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
                for (size_t t = 0; t < full.size(); ++t) {
                    if (t == 0 || full[t].first.first != full[t - 1].first.first) {
                        if (t > 0) seg_ptr.push_back(int64_t(seg_col.size()));
                        seg_q.push_back(k - 1);
                        seg_row.push_back(full[t].first.first);
                    }
                    seg_col.push_back(full[t].first.second);
                    seg_val.push_back(full[t].second);
                }
                if (!full.empty()) seg_ptr.push_back(int64_t(seg_col.size()));
            }
            d.nseg = int64_t(seg_q.size());
            {   // the constraints with a diagonal part, if few
                std::vector<int> dq;
                for (int q = 0; q < m; ++q)
                    for (int64_t i = 0; i < nds; ++i)
                        if (dmat[size_t(i) + size_t(nds) * q] != 0.0) {
                            dq.push_back(q);
                            break;
                        }
                if (int(dq.size()) <= kDqFew) {
                    d.ndq = int(dq.size());
                    dq_few.swap(dq);
                }
            }
        }
    }
    // aggregate pattern, full symmetric CSC with slots
    std::vector<int64_t> ag_cptr(n + 1, 0);
    std::vector<int> ag_row, ag_slot;
    {
        std::vector<std::vector<std::pair<int, int>>> cols(n);
        for (size_t t = 0; t < arow.size(); ++t) {
            int a = S.pos[arow[t]], c = S.pos[acol[t]];
            if (a < c) std::swap(a, c);
            const int sl = int(S.slot(a, c));
            cols[c].push_back({a, sl});
            if (a != c) cols[a].push_back({c, sl});
        }
        for (int j = 0; j < n; ++j) {
            std::sort(cols[j].begin(), cols[j].end());
            for (auto &p : cols[j]) {
                ag_row.push_back(p.first);
                ag_slot.push_back(p.second);
            }
            ag_cptr[j + 1] = int64_t(ag_row.size());
        }
    }
    // the same pattern by groups of 32 columns (row union and a slot per union row and
    // column) for the MFMA products X^ M
    const int nzg = (n + 31) / 32;
    std::vector<int64_t> zg_ptr(nzg + 1, 0);
    std::vector<int> zg_rows, zg_slot, zg_mma;
    for (int g = 0; g < nzg; ++g) {
        const int c0 = 32 * g, c1 = std::min(n, c0 + 32);
        std::vector<int> u;
        for (int c = c0; c < c1; ++c)
            for (int64_t t = ag_cptr[c]; t < ag_cptr[c + 1]; ++t) u.push_back(ag_row[t]);
        std::sort(u.begin(), u.end());
        u.erase(std::unique(u.begin(), u.end()), u.end());
        const int K = (int(u.size()) + 3) / 4 * 4;
        zg_mma.push_back(g);
        const size_t base = zg_slot.size();
        zg_slot.resize(base + size_t(K) * 32, -1);
        for (int k = 0; k < K; ++k) zg_rows.push_back(k < int(u.size()) ? u[k] : (u.empty() ? 0 : u.back()));
        for (int c = c0; c < c1; ++c)
            for (int64_t t = ag_cptr[c]; t < ag_cptr[c + 1]; ++t) {
                const int k = int(std::lower_bound(u.begin(), u.end(), ag_row[t]) - u.begin());
                zg_slot[base + size_t(k) * 32 + (c - c0)] = ag_slot[t];
            }
        zg_ptr[g + 1] = zg_ptr[g] + K;
    }
    // groups with a long union cut into pieces (split K; see kZmSplit)
    std::vector<int64_t> vg_ptr(1, 0);
    std::vector<int> vg_col, vg_piece, zs_g, zs_ptr(1, 0);
    int npiece = 0;
    for (int g = 0; g < nzg; ++g) {
        const int64_t a = zg_ptr[g], b = zg_ptr[g + 1];
        if (b - a > kZmSplit) {
            for (int64_t s = a; s < b; s += kZmPiece) {
                vg_ptr.push_back(std::min(b, s + kZmPiece));
                vg_col.push_back(g);
                vg_piece.push_back(npiece++);
            }
            zs_g.push_back(g);
            zs_ptr.push_back(npiece);
        } else {
            vg_ptr.push_back(b);
            vg_col.push_back(g);
            vg_piece.push_back(-1);
        }
    }
    zg_ptr.swap(vg_ptr);
    zg_mma.resize(vg_col.size());
    for (size_t v = 0; v < zg_mma.size(); ++v) zg_mma[v] = int(v);
    d.nzg = int(vg_col.size());
    d.nzg_mma = int(zg_mma.size());
    d.npiece = npiece;
    d.nzsplit = int(zs_g.size());
    // ---- uploads
    TRY(upload(h, &d.bl_first, S.bl_first));
    TRY(upload(h, &d.bl_rptr, S.bl_rptr));
    TRY(upload(h, &d.bl_rows, S.bl_rows));
    TRY(upload(h, &d.bl_off, S.bl_off));
    TRY(upload(h, &d.bl_subfirst, S.bl_subfirst));
    TRY(upload(h, &d.bl_fslot, fs));
    TRY(upload(h, &d.bl_bslot, bs));
    if (S.max_w <= 32 && S.max_h <= 64) {
        // the single-product walks' per-block row lists: row r at (r % 4) * 16 + r / 4
        std::vector<int> tfs(size_t(S.nb) * 64, -1), tfb(size_t(S.nb) * 64, -1), tbs(size_t(S.nb) * 64, -1);
        for (int b = 0; b < S.nb; ++b)
            for (int64_t t = S.bl_rptr[b]; t < S.bl_rptr[b + 1]; ++t) {
                const int r = int(t - S.bl_rptr[b]);
                const size_t idx = size_t(b) * 64 + size_t(r % 4) * 16 + size_t(r / 4);
                tfs[idx] = h->wslots.fwd[S.bl_rows[t]];
                tfb[idx] = h->wslots.birth[S.bl_rows[t]];
                tbs[idx] = h->wslots.bwd[S.bl_rows[t]];
            }
        TRY(upload(h, &d.wk_fs, tfs));
        TRY(upload(h, &d.wk_fb, tfb));
        TRY(upload(h, &d.wk_bs, tbs));
    }
    TRY(upload(h, &d.bl_dinv, dinv_off));
    TRY(upload(h, &d.up_ptr, up_ptr));
    TRY(upload(h, &d.up_pair, up_pair));
    TRY(upload(h, &d.up_slot, up_slot));
    TRY(upload(h, &d.su_rows, su_rows));
    TRY(upload(h, &d.wc_meta, wc_meta));
    TRY(upload(h, &d.wc_up, wc_up));
    TRY(upload(h, &d.col_block, S.col_block));
    TRY(upload(h, &d.slot_row, slot_row));
    TRY(upload(h, &d.slot_col, slot_col));
    TRY(upload(h, &d.cl_first, S.cl_first));
    TRY(upload(h, &d.cl_ptr, cl_ptr));
    TRY(upload(h, &d.cl_rows, cl_rows));
    TRY(upload(h, &d.cl_map_ptr, cl_map_ptr));
    TRY(upload(h, &d.cl_map, cl_map));
    TRY(upload(h, &d.wE, wE));
    TRY(upload(h, &d.asm_ptr, asm_ptr));
    TRY(upload(h, &d.asm_k, asm_k));
    TRY(upload(h, &d.asm_val, asm_val));
    TRY(upload(h, &d.con_ptr, con_ptr));
    TRY(upload(h, &d.con_pi, con_pi));
    TRY(upload(h, &d.con_pj, con_pj));
    TRY(upload(h, &d.con_slot, con_slot));
    TRY(upload(h, &d.con_val, con_val));
    {   // chunks of the long constraints (see kConLong)
        int64_t longest = 0;
        for (int k = 0; k < m; ++k) longest = std::max(longest, con_ptr[k + 2] - con_ptr[k + 1]);
        if (longest > kConLong) {
            std::vector<int> ch_con, ch_ptr(size_t(m) + 1, 0);
            std::vector<int64_t> ch_beg;
            for (int k = 0; k < m; ++k) {
                const int64_t len = con_ptr[k + 2] - con_ptr[k + 1];
                const int64_t nch = std::max<int64_t>(1, (len + kConChunk - 1) / kConChunk);
                for (int64_t c = 0; c < nch; ++c) {
                    ch_con.push_back(k);
                    ch_beg.push_back(con_ptr[k + 1] + c * kConChunk);
                }
                ch_ptr[k + 1] = int(ch_con.size());
            }
            d.con_chunks = int(ch_con.size());
            TRY(upload(h, &d.ch_con, ch_con));
            TRY(upload(h, &d.ch_beg, ch_beg));
            TRY(upload(h, &d.ch_ptr, ch_ptr));
        }
    }
    std::vector<double> bvec(prob->b, prob->b + m);
    TRY(upload(h, &d.b, bvec));
    TRY(upload(h, &d.had_pos, had_pos));
    TRY(upload(h, &d.had_val, had_val));
    TRY(upload(h, &d.kq_ptr, kq_ptr));
    TRY(upload(h, &d.kq_col, kq_col));
    TRY(upload(h, &d.aq_cptr, aq_cptr));
    TRY(upload(h, &d.aq_row, aq_row));
    TRY(upload(h, &d.aq_val, aq_val));
    d.nS = int64_t(S_col.size());
    TRY(upload(h, &d.S_rowptr, S_rowptr));
    TRY(upload(h, &d.S_col, S_col));
    TRY(upload(h, &d.am_ptr, am_ptr));
    TRY(upload(h, &d.am_sidx, am_sidx));
    TRY(upload(h, &d.am_val, am_val));
    TRY(upload(h, &d.ag_cptr, ag_cptr));
    TRY(upload(h, &d.ag_row, ag_row));
    TRY(upload(h, &d.ag_slot, ag_slot));
    TRY(upload(h, &d.zg_ptr, zg_ptr));
    TRY(upload(h, &d.zg_rows, zg_rows));
    TRY(upload(h, &d.zg_slot, zg_slot));
    TRY(upload(h, &d.zg_mma, zg_mma));
    TRY(upload(h, &d.zg_col, vg_col));
    TRY(upload(h, &d.zg_piece, vg_piece));
    TRY(upload(h, &d.zs_g, zs_g));
    TRY(upload(h, &d.zs_ptr, zs_ptr));
    if (d.npiece > 0) TRY(dalloc(h, &d.zpart, size_t(d.npiece) * 32 * size_t(n)));
    TRY(upload(h, &d.pos, S.pos));
    if (d.cc) {
        TRY(upload(h, &d.ccol, ccol));
        TRY(upload(h, &d.ucat, ucat));
        TRY(upload(h, &d.ds, ds_v));
        TRY(upload(h, &d.dmat, dmat));
        TRY(upload(h, &d.dq, dq_few));
        TRY(upload(h, &d.seg_q, seg_q));
        TRY(upload(h, &d.seg_row, seg_row));
        TRY(upload(h, &d.seg_ptr, seg_ptr));
        TRY(upload(h, &d.seg_col, seg_col));
        TRY(upload(h, &d.seg_val, seg_val));
    }
    // ---- workspace
    const size_t ns = size_t(S.nslot), nn = size_t(n) * n;
    h->ldb = int64_t(m) + 1;   // row m carries the SCE right-hand side through the factorisation
    TRY(dalloc(h, &h->X, ns));
    TRY(dalloc(h, &h->Xn, ns));
    TRY(dalloc(h, &h->Y, ns));
    TRY(dalloc(h, &h->G, ns));
    TRY(dalloc(h, &h->dX, ns));
    TRY(dalloc(h, &h->dY, ns));
    TRY(dalloc(h, &h->N, ns));
    TRY(dalloc(h, &h->Lhat, ns));
    TRY(dalloc(h, &h->z, size_t(m)));
    TRY(dalloc(h, &h->dz, size_t(m)));
    TRY(dalloc(h, &h->g, size_t(m)));
    TRY(dalloc(h, &h->hcol, size_t(m)));
    TRY(dalloc(h, &h->DinvN, size_t(dinv_off.back())));
    TRY(dalloc(h, &h->DinvL, size_t(dinv_off.back())));
    if (walk_g_ok(d)) {
        TRY(dalloc(h, &h->GN, size_t(d.nb) * 4096));
        TRY(dalloc(h, &h->GL, size_t(d.nb) * 4096));
    }
    if (h->prm.factorization == 1) {
        TRY(dalloc(h, &h->Dblk, size_t(dinv_off.back())));
        HIPCHK(h, hipMemsetAsync(h->Dblk, 0, size_t(dinv_off.back()) * sizeof(double), h->st));
    }
    TRY(dalloc(h, &h->Xh, nn));
    TRY(dalloc(h, &h->Yi, nn));
    TRY(dalloc(h, &h->W, nn));
    TRY(dalloc(h, &h->T, std::max<size_t>(size_t(d.nS), 1)));
    TRY(dalloc(h, &h->B, size_t(h->ldb) * std::max(m, 1)));
    TRY(dalloc(h, &h->pflags_b, size_t(potrf_flag_count(m))));
    TRY(dalloc(h, &h->pflags_f, size_t(potrf_flow_flag_count(m, m + 1))));
    TRY(dalloc(h, &h->pwork, potrf_work_doubles(m)));
    TRY(dalloc(h, &h->pwork_f, potrf_flow_work_doubles(m)));
    {
        double *blk = nullptr;   // flags | scal | alphas (kCand + 8 ints is a whole number of doubles)
        static_assert((kCand + 8) % 2 == 0, "flags must end on a double boundary");
        TRY(dalloc(h, &blk, size_t(kCand + 8) / 2 + 16 + kCand));
        h->flags = reinterpret_cast<int *>(blk);
        h->scal = blk + (kCand + 8) / 2;
        h->alphas = h->scal + 16;
        if (hipHostMalloc(reinterpret_cast<void **>(&h->rbh), kReadback, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            h->rbh = nullptr;
            return fail(h, SDPC_E_OOM, "pinned host allocation of the readback buffer failed");
        }
    }
    TRY(dalloc(h, &h->mwork, metrics_work_doubles(d)));
    TRY(dalloc(h, &h->alpha_cl, size_t(S.ncl)));
    TRY(dalloc(h, &h->alpha_hi, size_t(S.ncl)));
    TRY(dalloc(h, &h->cand, ns * kCand));
    TRY(dalloc(h, &h->ubuf, std::max<size_t>(size_t(d.nU), 1) * kCand));
    TRY(dalloc(h, &h->ydw, wave_chol_work_doubles(d)));
    TRY(dalloc(h, &h->ydw_dual, wave_chol_work_doubles(d)));
    TRY(dalloc(h, &h->part, std::max(size_t(2) * dX_chunks(d) * ns, size_t(rhs_had_parts(d)) * n)));
    if (d.cc) TRY(dalloc(h, &h->ccwork, cc_work_doubles(d)));
    HIPCHK(h, hipMemsetAsync(h->Lhat, 0, ns * sizeof(double), h->st));
    HIPCHK(h, hipMemsetAsync(h->N, 0, ns * sizeof(double), h->st));
    HIPCHK(h, hipMemsetAsync(h->flags, 0, (kCand + 8) * sizeof(int), h->st));
    HIPCHK(h, hipMemsetAsync(h->pflags_b, 0, potrf_flag_count(m) * sizeof(int), h->st));
    HIPCHK(h, hipMemsetAsync(h->pflags_f, 0, potrf_flow_flag_count(m, m + 1) * sizeof(int), h->st));
    for (auto &e : h->ev) HIPCHK(h, hipEventCreate(&e));
    for (auto &set : h->evs)
        for (auto &e : set) HIPCHK(h, hipEventCreate(&e));
    HIPCHK(h, hipEventCreateWithFlags(&h->ev_rb, hipEventDisableTiming));
    HIPCHK(h, hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
    HIPCHK(h, hipEventCreateWithFlags(&h->ev_dy, hipEventDisableTiming));
    HIPCHK(h, hipEventCreateWithFlags(&h->ev_dual, hipEventDisableTiming));
    launch_init_point(d, h->prm.lambda0, h->X, h->Y, h->z, h->st);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipStreamSynchronize(h->st));
    return SDPC_OK;
}

sdpc_status sdpc_analyze(const sdpc_problem *prob, const sdpc_params *params, sdpc_analysis *info, int32_t *perm,
                         int64_t *cptr, int32_t *cidx, int32_t *nS) {
    if (!prob || !info || !prob->ptr || prob->n <= 0 || prob->m < 0 || (prob->m > 0 && !prob->b)) return SDPC_E_ARG;
    if (prob->ptr[prob->m + 1] > 0 && (!prob->row || !prob->col || !prob->val)) return SDPC_E_ARG;
    std::unique_ptr<sdpc_handle> h(new (std::nothrow) sdpc_handle());
    if (!h) return SDPC_E_OOM;
    h->n = prob->n;
    h->m = prob->m;
    h->prm = params ? *params : sdpc_default_params();
    sdpc_status s = check_problem(prob, h.get());
    std::vector<int> arow, acol;
    if (s == SDPC_OK) s = analyze_impl(prob, h.get(), arow, acol);
    if (s != SDPC_OK) {
        if (h->prm.verbose) fprintf(stderr, "sdpc_analyze: %s\n", h->err.c_str());
        return s;
    }
    const Symbolic &S = h->S;
    std::memset(info, 0, sizeof(*info));
    info->nslot = S.nslot;
    for (uint8_t e : S.isE) info->nnzE += e;
    info->ncliques = S.ncl;
    info->nblocks = S.nb;
    info->max_clique = S.max_clique;
    info->max_block_rows = S.max_h;
    info->max_block_cols = S.max_w;
    info->nfwd = h->slots.nfwd;
    info->nbwd = h->slots.nbwd;
    bool had = prob->m > 0;
    for (int k = 1; k <= prob->m && had; ++k) {
        int p0 = -1;
        bool any = false;
        for (int64_t t = prob->ptr[k]; t < prob->ptr[k + 1]; ++t) {
            if (prob->val[t] == 0.0) continue;
            if (prob->row[t] != prob->col[t] || (p0 >= 0 && prob->row[t] != p0)) { had = false; break; }
            p0 = prob->row[t];
            any = true;
        }
        had = had && any;
    }
    info->hadamard = had ? 1 : 0;
    int64_t off = 0;
    if (cptr) cptr[0] = 0;
    for (int r = 0; r < S.ncl; ++r) {
        const int f = S.cl_first[r];
        for (int64_t t = S.sptr[f]; t < S.sptr[f + 1]; ++t) {
            if (cidx) cidx[off] = S.perm[S.sidx[t]];
            ++off;
        }
        if (cptr) cptr[r + 1] = off;
        if (nS) nS[r] = S.cl_first[r + 1] - f;
    }
    info->sum_clique = off;
    info->limit_clique = kMaxClique;
    info->limit_panel = kMaxPanel;
    info->limit_m = kMaxM;
    {
        const int64_t n = prob->n, m = prob->m, ns = S.nslot;
        info->device_bytes = int64_t(sizeof(double)) * (3 * n * n + (m + 1) * std::max<int64_t>(m, 1) +
                                                         (kCand + 12) * ns + int64_t(S.nb) * 4 * 64 * 32);
    }
    if (perm) std::copy(S.perm.begin(), S.perm.end(), perm);
    return SDPC_OK;
}

sdpc_status sdpc_create(const sdpc_problem *prob, const sdpc_params *params, hipStream_t stream, sdpc_handle **out) {
    if (!out) return SDPC_E_ARG;
    *out = nullptr;
    if (!prob || !prob->ptr || prob->n <= 0 || prob->m < 0 || (prob->m > 0 && !prob->b)) return SDPC_E_ARG;
    if (prob->ptr[prob->m + 1] > 0 && (!prob->row || !prob->col || !prob->val)) return SDPC_E_ARG;
    sdpc_handle *h = new (std::nothrow) sdpc_handle();
    if (!h) return SDPC_E_OOM;
    sdpc_status s = create_impl(prob, params, stream, h);
    if (s != SDPC_OK) {
        // keep the message reachable for the caller through stderr only; the handle is gone
        if (h->prm.verbose) fprintf(stderr, "sdpc_create: %s\n", h->err.c_str());
        sdpc_destroy(h);
        return s;
    }
    *out = h;
    return SDPC_OK;
}

}  // extern "C"

namespace {

int read_flag(sdpc_handle *h, int idx) {
    int v = 0;
    (void)hipMemcpy(&v, h->flags + idx, sizeof(int), hipMemcpyDeviceToHost);
    return v;
}

// Y = N N^T; Lhat (Algorithm 1); X^ and Y^{-1}; B lower; optional Cholesky of B.
// Flags of the phases, checked after the launch sequence has completed.
// fl_read: the 8 phase flags flags[kCand .. kCand + 8) as already read back, or null
// to read them here.
sdpc_status check_flags(sdpc_handle *h, bool potrf, const int *fl_read = nullptr) {
    int fl[8];
    if (fl_read)
        std::memcpy(fl, fl_read, sizeof(fl));
    else
        HIPCHK(h, hipMemcpy(fl, h->flags + kCand, sizeof(fl), hipMemcpyDeviceToHost));
    if (fl[5])
        return fail(h, SDPC_E_NOT_PD, "Y is not positive definite (storage block " + std::to_string(fl[5] - 1) + ")");
    if (fl[1])
        return fail(h, SDPC_E_NOT_PD, "clique block of Xbar not positive definite (clique " + std::to_string(fl[1] - 1) + ")");
    if (fl[3])
        return fail(h, SDPC_E_NOT_PD, "clique block of the updated Xbar not positive definite (clique " +
                                          std::to_string(fl[3] - 1) + ")");
    if (fl[0] || fl[4]) return fail(h, SDPC_E_NOT_PD, "singular diagonal block in a factor");
    if (potrf && fl[2] < 0) return fail(h, SDPC_E_HIP, "SCE solve: an internal hand-over wait ran out");
    if (potrf && fl[2])
        return fail(h, SDPC_E_NOT_PD, "Schur complement matrix not positive definite at pivot " + std::to_string(fl[2] - 1));
    return SDPC_OK;
}

void read_scm_timing(sdpc_handle *h, int set) {
    for (int i = 0; i < 5; ++i) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, h->evs[set][i], h->evs[set][i + 1]);
        h->scm_ms[i] = ms;
    }
}

// SCM Cholesky of the leading m columns of B with rows m .. rows - 1 riding along,
// in the form the parameters choose; fail: pivot + 1, or -1 if a hand-over wait ran out.
void potrf_rows(sdpc_handle *h, int m, int rows, double *B, int64_t ldb, int *fail) {
    if (h->prm.chol_kernel == 0)
        launch_potrf_flow(m, rows, B, ldb, h->pflags_f, h->pwork_f, ++h->epoch_f, fail, h->st);
    else
        launch_potrf_rows(m, rows, B, ldb, h->pwork, fail, h->st);
}

// The factor X^ is applied through, from Xbar: Lhat of Algorithm 1 (X^{-1} = Lhat
// Lhat^T), or with factorization 1 the unit-lower L^{-1} and the block diagonal D of
// X^ = L^T D L (eq. sparse_fact); then the inverses of the factor's diagonal blocks.
void launch_xside(sdpc_handle *h, const double *Xbar, int *fail_clique, int *fail_dinv) {
    if (h->prm.factorization == 1)
        launch_ldl_cliques(h->d, Xbar, h->Lhat, h->Dblk, fail_clique, h->st);
    else
        launch_algorithm1(h->d, Xbar, h->Lhat, fail_clique, h->st);
    launch_dinv(h->d, h->Lhat, h->DinvL, fail_dinv, h->st, h->GL, h->Dblk);
}

// Y = N N^T; Lhat (Algorithm 1); X^ and Y^{-1}; B lower; optional Cholesky of B.
// Inside an iteration (in_step) the factor of Y may come from the dual step, the
// X side may already have been formed at the end of the previous iteration, and
// nothing is synchronised: the caller checks the flags once at its end.  With
// twin_on_device the factor of Y is the dual step's twin whose index the dual
// step left in alphas[3] (the next iteration's phase, enqueued before the host
// knows the index; if there is none, N is stale and the caller discards the phase).
sdpc_status scm_phase(sdpc_handle *h, const double *Xbar, const double *Y, double *B, int64_t ldb, bool factor,
                      bool in_step = false, bool twin_on_device = false) {
    DevStruct &d = h->d;
    hipStream_t st = h->st;
    const bool xready = in_step && h->xside_ready;
    if (!(in_step && h->flags_zeroed)) HIPCHK(h, hipMemsetAsync(h->flags, 0, (kCand + 8) * sizeof(int), st));
    h->flags_zeroed = false;
    h->scm_ready = false;
    h->evs_set ^= 1;
    hipEvent_t *evs = h->evs[h->evs_set];
    HIPCHK(h, hipEventRecord(evs[0], st));
    if (twin_on_device)
        launch_copy_selected(d.nslot, h->cand, h->alphas + 3, kCand, h->N, st);
    else if (in_step && h->next_cand >= 0)   // N = the dual step's twin factor of this Y
        HIPCHK(h, hipMemcpyAsync(h->N, h->cand + size_t(h->next_cand) * size_t(d.nslot),
                                 size_t(d.nslot) * sizeof(double), hipMemcpyDeviceToDevice, st));
    else
        launch_sn_chol(d, Y, h->N, h->ubuf, h->ydw, h->flags + kCand + 5, st);
    h->next_cand = -1;
    launch_dinv(d, h->N, h->DinvN, h->flags + kCand, st, h->GN);
    HIPCHK(h, hipEventRecord(evs[1], st));
    if (!xready) launch_xside(h, Xbar, h->flags + kCand + 1, h->flags + kCand);
    HIPCHK(h, hipEventRecord(evs[2], st));
    // Y^{-1} and X^ in one launch: the two walks are latency-bound and fill each
    // other's idle compute units
    launch_inverse_by_solves(d, h->N, h->DinvN, h->Yi, h->Lhat, h->DinvL, h->Xh, st, nullptr, h->Dblk, h->GN,
                             h->GL);
    h->xside_ready = false;
    HIPCHK(h, hipEventRecord(evs[3], st));
    if (d.hadamard)
        launch_scm_hadamard(d, h->Xh, h->Yi, B, ldb, st);
    else if (d.cc)
        launch_scm_cc(d, h->Xh, h->Yi, h->W, h->ccwork, B, ldb, st);
    else
        launch_scm_general(d, h->kq_ptr_h.data(), h->Xh, h->Yi, h->W, h->T, B, ldb, st);
    HIPCHK(h, hipEventRecord(evs[4], st));
    if (factor) potrf_rows(h, d.m, d.m, B, ldb, h->flags + kCand + 2);
    HIPCHK(h, hipEventRecord(evs[5], st));
    HIPCHK(h, hipGetLastError());
    if (in_step) return SDPC_OK;
    HIPCHK(h, hipStreamSynchronize(st));
    read_scm_timing(h, h->evs_set);
    return check_flags(h, factor);
}

double since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Largest alpha in (0, 1] with Y + alpha dY positive definite (parallel candidate
// tests), enqueued on the side stream once dY is ready; the caller joins ev_dual
// on the main stream before reading the result (bracket[0]).
sdpc_status dual_step_launch(sdpc_handle *h) {
    HIPCHK(h, hipEventRecord(h->ev_dy, h->st));
    HIPCHK(h, hipStreamWaitEvent(h->side, h->ev_dy, 0));
    launch_dual_step(h->d, h->Y, h->dY, h->dual_rounds, h->dual_test, h->prm.gamma, h->cand, h->ubuf, h->ydw_dual,
                     h->flags, h->alphas, h->side);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipEventRecord(h->ev_dual, h->side));
    return SDPC_OK;
}

struct IterInfo {
    bool stop = false;
    double pobj, dobj, relgap, pinf, dinf, mu, beta;
};

sdpc_status read_metrics(sdpc_handle *h, IterInfo &it) {
    DevStruct &d = h->d;
    double sc[8];
    if (h->metrics_ready) {   // formed and read back with the previous step
        std::memcpy(sc, h->msc, sizeof(sc));
        h->metrics_ready = false;
    } else {
        launch_metrics(d, h->X, h->Y, h->z, h->G, h->scal, h->mwork, h->st);
        HIPCHK(h, hipGetLastError());
        HIPCHK(h, hipMemcpyAsync(sc, h->scal, 6 * sizeof(double), hipMemcpyDeviceToHost, h->st));
        HIPCHK(h, hipStreamSynchronize(h->st));
    }
    if (sc[5] != 0.0) return fail(h, SDPC_E_NUMERIC, "non-finite iterate");
    it.pobj = sc[0];
    it.dobj = sc[1];
    it.relgap = std::fabs(sc[0] - sc[1]) / std::max(1.0, (std::fabs(sc[0]) + std::fabs(sc[1])) / 2.0);
    it.pinf = sc[2] / (1.0 + h->bmax);
    it.dinf = sc[3] / (1.0 + h->a0max);
    it.mu = sc[4] / h->n;
    const bool feas = it.pinf <= h->prm.feas_tol && it.dinf <= h->prm.feas_tol;
    it.beta = feas ? h->prm.beta_feas : h->prm.beta_infeas;
    it.stop = it.relgap <= h->prm.gap_tol && feas;
    return SDPC_OK;
}

void fill_result(sdpc_handle *h, const IterInfo &it, sdpc_result *res) {
    if (!res) return;
    res->iters = h->iters;
    res->pobj = it.pobj;
    res->dobj = it.dobj;
    res->rel_gap = it.relgap;
    res->pinf = it.pinf;
    res->dinf = it.dinf;
    res->mu = it.mu;
    res->beta = it.beta;
    res->alpha_p = h->last_alpha[0];
    res->alpha_d = h->last_alpha[1];
    res->device_bytes = h->bytes;
}

// One iteration.  *done = true when the stopping test held (no update).  With
// mu_target > 0 the step is a centring step instead: the direction aims at the
// point of the central path with X Y = mu_target I (the target beta mu of Step 2
// replaced by mu_target), and the stopping test is not applied.
sdpc_status step_impl(sdpc_handle *h, sdpc_result *res, bool *done, double mu_target = 0.0) {
    DevStruct &d = h->d;
    hipStream_t st = h->st;
    IterInfo it;
    TRY(read_metrics(h, it));
    *done = it.stop && !(mu_target > 0.0);
    if (*done) {
        fill_result(h, it, res);
        return SDPC_OK;
    }
    const double bm = (mu_target > 0.0) ? mu_target : it.beta * it.mu;
    if (!h->scm_ready) TRY(scm_phase(h, h->X, h->Y, h->B, h->ldb, false, true));
    h->scm_ready = false;
    const int evs_set = h->evs_set;
    hipEvent_t *ev = h->ev;
    HIPCHK(h, hipEventRecord(ev[0], st));
    // right-hand side: g = b - beta mu A(Y^{-1}) + A(X^ G Y^{-1})
    if (d.hadamard)
        launch_rhs_hadamard(d, h->G, h->Xh, h->Yi, h->part, h->hcol, st);
    else if (d.cc)
        launch_scm_cc_extra_column(d, h->G, h->Xh, h->Yi, h->W, h->ccwork, h->hcol, st);
    else
        launch_scm_extra_column(d, h->G, h->Xh, h->Yi, h->W, h->T, h->hcol, st);
    launch_rhs(d, h->Yi, h->hcol, bm, h->g, h->mwork, st);
    HIPCHK(h, hipEventRecord(ev[1], st));
    HIPCHK(h, hipMemsetAsync(h->flags + kCand + 2, 0, sizeof(int), st));
    launch_set_row(d.m, h->g, h->B + d.m, h->ldb, st);
    potrf_rows(h, d.m, d.m + 1, h->B, h->ldb, h->flags + kCand + 2);
    HIPCHK(h, hipEventRecord(ev[6], st));
    launch_potrs_bwd(d.m, h->B, h->ldb, h->B + d.m, h->ldb, h->dz, h->pflags_b, ++h->epoch, h->flags + kCand + 2, st);
    HIPCHK(h, hipEventRecord(ev[2], st));
    // dY = G - sum dz_k A_k; the dual step runs on the side stream while dX on E and
    // the clique-wise primal step run here
    launch_assemble(d, h->dz, 0.0, 1.0, h->G, h->dY, st);
    TRY(dual_step_launch(h));
    launch_zcol(d, h->Xh, h->dY, h->W, st);
    launch_dX_blocked(d, h->W, h->Yi, h->X, bm, h->part, h->dX, st);
    launch_alpha_cliques(d, h->X, h->dX, h->alpha_cl, h->alpha_hi, h->scal + 8, st);
    // Step 4 for X with alpha_p still on the device, into Xn (X itself is replaced
    // only once the iteration is known to have succeeded), then Algorithm 1 and
    // Lhat's diagonal inverses for the next iteration while the dual step runs
    const double gm = h->prm.gamma;
    launch_axpy_checked(d.nslot, h->X, h->dX, h->scal + 8, nullptr, gm, nullptr, 0, h->Xn, st);
    launch_xside(h, h->Xn, h->flags + kCand + 3, h->flags + kCand + 4);
    HIPCHK(h, hipStreamWaitEvent(st, h->ev_dual, 0));   // join the dual step
    HIPCHK(h, hipEventRecord(ev[3], st));   // both step lengths are known
    // Step 4 for Y and z (alpha_d = bracket[0] on the device; the same fma as the
    // dual step's twin candidates, whose factor of the new Y is then reused).  If a
    // factorisation of this iteration reported a failure (flags kCand .. kCand + 5)
    // or a step length is zero, Y and z stay as they are.
    launch_axpy_checked(d.nslot, h->Y, h->dY, h->alphas, h->scal + 8, gm, h->flags + kCand, 6, h->Y, st);
    launch_axpy_checked(d.m, h->z, h->dz, h->alphas, h->scal + 8, gm, h->flags + kCand, 6, h->z, st);
    // the metrics of the new iterate (Step 1 of the next iteration), read back with
    // the step lengths and the flags: one synchronisation per iteration
    launch_metrics(d, h->Xn, h->Y, h->z, h->G, h->scal, h->mwork, st);
    HIPCHK(h, hipGetLastError());
    // (one copy into pinned memory; the flags are cleared behind it for the next
    // iteration, so that its first operation is a kernel)
    HIPCHK(h, hipMemcpyAsync(h->rbh, h->flags + kCand, kReadback, hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipMemsetAsync(h->flags, 0, (kCand + 8) * sizeof(int), st));
    HIPCHK(h, hipEventRecord(h->ev_rb, st));
    h->flags_zeroed = true;
    // Behind the readback, the next iteration's Schur complement phase, on the
    // assumption that this iteration succeeds and the dual step leaves the factor
    // of the new Y (the X side of the new X is already formed): the device goes
    // on while the host reads the step back.  It writes only the factor of Y and
    // its diagonal inverses, X^, Y^{-1}, B and the assembly's work space, which
    // the next iteration recomputes if the assumption fails.  Skipped near the
    // stopping test, where the next iteration is likely not to run.
    const bool ahead = (mu_target > 0.0) || !(it.relgap <= kAheadGap * h->prm.gap_tol);
    if (ahead) {
        h->xside_ready = true;   // Lhat of Xn is enqueued above
        TRY(scm_phase(h, h->Xn, h->Y, h->B, h->ldb, false, true, true));
    }
    HIPCHK(h, hipEventSynchronize(h->ev_rb));
    int fl[8];
    double sc[16], br[4];
    std::memcpy(fl, h->rbh, sizeof(fl));
    std::memcpy(sc, h->rbh + sizeof(fl), sizeof(sc));
    std::memcpy(br, h->rbh + sizeof(fl) + sizeof(sc), sizeof(br));
    std::memcpy(h->msc, sc, sizeof(h->msc));
    const double ap = sc[8];
    read_scm_timing(h, evs_set);
    TRY(check_flags(h, true, fl));
    const double t_scm = h->scm_ms[0] + h->scm_ms[1] + h->scm_ms[2] + h->scm_ms[3];
    float ms_rhs = 0, ms_chol = 0, ms_pm = 0, ms_potrf = 0;
    (void)hipEventElapsedTime(&ms_potrf, ev[1], ev[6]);
    (void)hipEventElapsedTime(&ms_rhs, ev[0], ev[1]);
    (void)hipEventElapsedTime(&ms_chol, ev[1], ev[2]);
    (void)hipEventElapsedTime(&ms_pm, ev[2], ev[3]);
    const double ad = br[0];
    const double ms_ad = 0.0;   // inside ms_pm: the dual step overlaps dX, alpha_p and the next X side
    h->last_alpha[0] = ap;
    h->last_alpha[1] = ad;
    if (!(ap > 0.0) || !(ad > 0.0)) return fail(h, SDPC_E_STAGNATION, "step length collapsed to zero");
    // the iteration succeeded: the new X, the metrics, Lhat and the factor of the new Y
    // held by a dual-step twin all belong to the new iterate
    std::swap(h->X, h->Xn);
    h->metrics_ready = true;
    h->xside_ready = true;
    h->next_cand = (br[3] >= 0.0) ? int(br[3]) : -1;
    if (ahead && h->next_cand >= 0) {   // the phase enqueued ahead belongs to the new iterate
        h->scm_ready = true;
        h->next_cand = -1;
    }
    h->iters++;
    if (res) {
        res->t_scm_ms += t_scm + ms_rhs;
        res->t_chol_ms += ms_chol;
        res->t_pmatrix_ms += ms_pm + ms_ad;
        res->t_potrf_ms += ms_potrf;
        res->n_potrf += 1;
    }
    fill_result(h, it, res);
    if (h->prm.verbose)
        fprintf(stderr,
                "it %3d pobj %+.10e dobj %+.10e gap %.2e pinf %.2e dinf %.2e mu %.2e ap %.4f ad %.4f "
                "scm %.3f chol %.3f pm %.3f ad %.3f ms\n",
                h->iters, it.pobj, it.dobj, it.relgap, it.pinf, it.dinf, it.mu, ap, ad, t_scm + ms_rhs, ms_chol,
                ms_pm, ms_ad);
    return SDPC_OK;
}

}  // namespace

extern "C" {

sdpc_status sdpc_reset(sdpc_handle *h) {
    if (!h) return SDPC_E_ARG;
    launch_init_point(h->d, h->prm.lambda0, h->X, h->Y, h->z, h->st);
    HIPCHK(h, hipGetLastError());
    h->iters = 0;
    h->next_cand = -1;
    h->xside_ready = false;
    h->metrics_ready = false;
    h->scm_ready = false;
    return SDPC_OK;
}

sdpc_status sdpc_step(sdpc_handle *h, sdpc_result *res) {
    if (!h) return SDPC_E_ARG;
    if (res) std::memset(res, 0, sizeof(*res));
    const auto t0 = std::chrono::steady_clock::now();
    bool done = false;
    sdpc_status s = step_impl(h, res, &done);
    if (res) {
        res->status = s;
        res->t_total_ms = since(t0);
    }
    return s;
}

sdpc_status sdpc_solve(sdpc_handle *h, sdpc_result *res) {
    if (!h) return SDPC_E_ARG;
    sdpc_result r;
    std::memset(&r, 0, sizeof(r));
    const auto t0 = std::chrono::steady_clock::now();
    sdpc_status s = sdpc_reset(h);
    bool done = false;
    while (s == SDPC_OK) {
        s = step_impl(h, &r, &done);
        if (s != SDPC_OK || done) break;
        if (h->iters >= h->prm.max_iter) {
            IterInfo it;
            s = read_metrics(h, it);
            if (s == SDPC_OK) {
                fill_result(h, it, &r);
                s = it.stop ? SDPC_OK : fail(h, SDPC_E_MAXITER, "iteration limit reached");
            }
            break;
        }
    }
    r.status = s;
    r.iters = h->iters;
    r.t_total_ms = since(t0);
    r.device_bytes = h->bytes;
    if (res) *res = r;
    return s;
}

sdpc_status sdpc_scm(sdpc_handle *h, const double *d_Xbar_E, const double *d_Y_E, double *d_B, int64_t ldb,
                     int32_t factor) {
    if (!h || !d_Xbar_E || !d_Y_E || !d_B || ldb < h->m) return h ? fail(h, SDPC_E_ARG, "bad sdpc_scm arguments") : SDPC_E_ARG;
    return scm_phase(h, d_Xbar_E, d_Y_E, d_B, ldb, factor != 0);
}

sdpc_status sdpc_potrf(sdpc_handle *h, double *d_B, int64_t ldb, int32_t m) {
    if (!h || !d_B || m < 0 || ldb < m || m > h->m) return h ? fail(h, SDPC_E_ARG, "bad sdpc_potrf arguments") : SDPC_E_ARG;
    h->flags_zeroed = false;
    HIPCHK(h, hipMemsetAsync(h->flags + kCand + 2, 0, sizeof(int), h->st));
    potrf_rows(h, m, m, d_B, ldb, h->flags + kCand + 2);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipStreamSynchronize(h->st));
    const int f = read_flag(h, kCand + 2);
    if (f < 0) return fail(h, SDPC_E_HIP, "internal hand-over wait ran out");
    if (f) return fail(h, SDPC_E_NOT_PD, "matrix not positive definite at pivot " + std::to_string(f - 1));
    return SDPC_OK;
}

sdpc_status sdpc_get_pattern(const sdpc_handle *h, int64_t *nslot, int32_t *iE, int32_t *jE, int32_t *perm,
                             int32_t *ncliques) {
    if (!h) return SDPC_E_ARG;
    if (nslot) *nslot = h->S.nslot;
    if (iE || jE)
        for (int64_t s = 0; s < h->S.nslot; ++s) {
            const int r = h->slot_row_h[s], c = h->slot_col_h[s];
            if (iE) iE[s] = r >= 0 ? h->S.perm[r] : -1;
            if (jE) jE[s] = c >= 0 ? h->S.perm[c] : -1;
        }
    if (perm) std::copy(h->S.perm.begin(), h->S.perm.end(), perm);
    if (ncliques) *ncliques = h->S.ncl;
    return SDPC_OK;
}

sdpc_status sdpc_get_cliques(const sdpc_handle *h, int64_t *cptr, int32_t *cidx, int32_t *nS) {
    if (!h) return SDPC_E_ARG;
    const Symbolic &S = h->S;
    int64_t off = 0;
    if (cptr) cptr[0] = 0;
    for (int r = 0; r < S.ncl; ++r) {
        const int f = S.cl_first[r];
        for (int64_t t = S.sptr[f]; t < S.sptr[f + 1]; ++t) {
            if (cidx) cidx[off] = S.perm[S.sidx[t]];
            ++off;
        }
        if (cptr) cptr[r + 1] = off;
        if (nS) nS[r] = S.cl_first[r + 1] - f;
    }
    return SDPC_OK;
}

sdpc_status sdpc_get_solution(const sdpc_handle *hc, double *d_Xbar_E, double *d_Y_E, double *d_z) {
    sdpc_handle *h = const_cast<sdpc_handle *>(hc);
    if (!h) return SDPC_E_ARG;
    const size_t ns = size_t(h->S.nslot) * sizeof(double);
    if (d_Xbar_E) HIPCHK(h, hipMemcpyAsync(d_Xbar_E, h->X, ns, hipMemcpyDeviceToDevice, h->st));
    if (d_Y_E) HIPCHK(h, hipMemcpyAsync(d_Y_E, h->Y, ns, hipMemcpyDeviceToDevice, h->st));
    if (d_z) HIPCHK(h, hipMemcpyAsync(d_z, h->z, size_t(h->m) * sizeof(double), hipMemcpyDeviceToDevice, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    return SDPC_OK;
}

sdpc_status sdpc_set_state(sdpc_handle *h, const double *d_Xbar_E, const double *d_Y_E, const double *d_z) {
    if (!h || !d_Xbar_E || !d_Y_E || !d_z) return h ? fail(h, SDPC_E_ARG, "null state pointer") : SDPC_E_ARG;
    const size_t ns = size_t(h->S.nslot) * sizeof(double);
    HIPCHK(h, hipMemcpyAsync(h->X, d_Xbar_E, ns, hipMemcpyDeviceToDevice, h->st));
    HIPCHK(h, hipMemcpyAsync(h->Y, d_Y_E, ns, hipMemcpyDeviceToDevice, h->st));
    HIPCHK(h, hipMemcpyAsync(h->z, d_z, size_t(h->m) * sizeof(double), hipMemcpyDeviceToDevice, h->st));
    launch_mask_E(h->d, h->X, h->st);
    launch_mask_E(h->d, h->Y, h->st);
    HIPCHK(h, hipGetLastError());
    h->next_cand = -1;
    h->xside_ready = false;
    h->metrics_ready = false;
    h->scm_ready = false;
    return SDPC_OK;
}

sdpc_status sdpc_get_factors(const sdpc_handle *hc, double *d_N, double *d_Lhat) {
    sdpc_handle *h = const_cast<sdpc_handle *>(hc);
    if (!h) return SDPC_E_ARG;
    const size_t ns = size_t(h->S.nslot) * sizeof(double);
    if (d_N) HIPCHK(h, hipMemcpyAsync(d_N, h->N, ns, hipMemcpyDeviceToDevice, h->st));
    if (d_Lhat) HIPCHK(h, hipMemcpyAsync(d_Lhat, h->Lhat, ns, hipMemcpyDeviceToDevice, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    return SDPC_OK;
}

sdpc_status sdpc_get_dense(const sdpc_handle *hc, double *d_Xhat, double *d_Yinv) {
    sdpc_handle *h = const_cast<sdpc_handle *>(hc);
    if (!h) return SDPC_E_ARG;
    const size_t nn = size_t(h->n) * h->n * sizeof(double);
    if (d_Xhat) HIPCHK(h, hipMemcpyAsync(d_Xhat, h->Xh, nn, hipMemcpyDeviceToDevice, h->st));
    if (d_Yinv) HIPCHK(h, hipMemcpyAsync(d_Yinv, h->Yi, nn, hipMemcpyDeviceToDevice, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    return SDPC_OK;
}

sdpc_status sdpc_get_direction(const sdpc_handle *hc, double *d_dz, double *d_dX_E, double *d_dY_E, double *alpha) {
    sdpc_handle *h = const_cast<sdpc_handle *>(hc);
    if (!h) return SDPC_E_ARG;
    const size_t ns = size_t(h->S.nslot) * sizeof(double);
    if (d_dz) HIPCHK(h, hipMemcpyAsync(d_dz, h->dz, size_t(h->m) * sizeof(double), hipMemcpyDeviceToDevice, h->st));
    if (d_dX_E) HIPCHK(h, hipMemcpyAsync(d_dX_E, h->dX, ns, hipMemcpyDeviceToDevice, h->st));
    if (d_dY_E) HIPCHK(h, hipMemcpyAsync(d_dY_E, h->dY, ns, hipMemcpyDeviceToDevice, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    if (alpha) {
        alpha[0] = h->last_alpha[0];
        alpha[1] = h->last_alpha[1];
    }
    return SDPC_OK;
}

sdpc_status sdpc_complete_dense(sdpc_handle *h, double *d_Xhat) {
    if (!h) return SDPC_E_ARG;
    DevStruct &d = h->d;
    hipStream_t st = h->st;
    h->flags_zeroed = false;
    h->scm_ready = false;
    HIPCHK(h, hipMemsetAsync(h->flags + kCand, 0, 8 * sizeof(int), st));
    h->xside_ready = false;
    launch_xside(h, h->X, h->flags + kCand + 1, h->flags + kCand);
    launch_inverse_by_solves(d, h->Lhat, h->DinvL, h->Xh, nullptr, nullptr, nullptr, st, h->Dblk, h->GL);
    if (d_Xhat) launch_unpermute(d, h->Xh, d_Xhat, st);
    HIPCHK(h, hipGetLastError());
    int fl[2] = {0, 0};
    HIPCHK(h, hipMemcpyAsync(fl, h->flags + kCand, sizeof(fl), hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipStreamSynchronize(st));
    if (fl[1])
        return fail(h, SDPC_E_NOT_PD, "clique block of Xbar not positive definite (clique " + std::to_string(fl[1] - 1) + ")");
    if (fl[0]) return fail(h, SDPC_E_NOT_PD, "singular diagonal block in a factor");
    h->xside_ready = true;   // Lhat and its diagonal inverses belong to the current X
    return SDPC_OK;
}

sdpc_status sdpc_center(sdpc_handle *h, double mu, int32_t max_steps, double tol, int32_t *steps,
                        double *last_rel_step) {
    if (!h || !(mu > 0.0) || !std::isfinite(mu) || max_steps < 1 || !(tol >= 0.0))
        return h ? fail(h, SDPC_E_ARG, "bad sdpc_center arguments (need mu > 0, max_steps >= 1, tol >= 0)")
                 : SDPC_E_ARG;
    const int m = h->m;
    std::vector<double> dz(size_t(std::max(m, 1))), z(size_t(std::max(m, 1)));
    sdpc_status s = SDPC_OK;
    double rel = INFINITY;
    int k = 0;
    while (k < max_steps) {
        bool done = false;
        s = step_impl(h, nullptr, &done, mu);
        if (s != SDPC_OK) break;
        ++k;
        // how far z moved: gamma alpha_d dz relative to z
        if (m > 0) {
            HIPCHK(h, hipMemcpy(dz.data(), h->dz, size_t(m) * sizeof(double), hipMemcpyDeviceToHost));
            HIPCHK(h, hipMemcpy(z.data(), h->z, size_t(m) * sizeof(double), hipMemcpyDeviceToHost));
        }
        double mdz = 0.0, mz = 1.0;
        for (int i = 0; i < m; ++i) {
            mdz = std::max(mdz, std::fabs(dz[i]));
            mz = std::max(mz, std::fabs(z[i]));
        }
        rel = h->prm.gamma * h->last_alpha[1] * mdz / mz;
        if (rel <= tol) break;
    }
    if (steps) *steps = k;
    if (last_rel_step) *last_rel_step = rel;
    return s;
}

sdpc_status sdpc_adjoint(sdpc_handle *h, const double *d_GL_E, const double *d_dLdz, double *d_gb,
                         double *d_gC_E) {
    if (!h || !d_GL_E || !d_gb || !d_gC_E) return h ? fail(h, SDPC_E_ARG, "bad sdpc_adjoint arguments") : SDPC_E_ARG;
    DevStruct &d = h->d;
    hipStream_t st = h->st;
    const int m = d.m;
    // B, X^ and Y^{-1} of the current iterate
    TRY(scm_phase(h, h->X, h->Y, h->B, h->ldb, false));
    // h_p = A_p . (X^ G_L Y^{-1}), then lambda = B^{-1} (h + dL/dz) by the SCM Cholesky
    // with the right-hand side riding along as row m, and the backward substitution
    if (d.hadamard)
        launch_rhs_hadamard(d, d_GL_E, h->Xh, h->Yi, h->part, h->hcol, st);
    else if (d.cc)
        launch_scm_cc_extra_column(d, d_GL_E, h->Xh, h->Yi, h->W, h->ccwork, h->hcol, st);
    else
        launch_scm_extra_column(d, d_GL_E, h->Xh, h->Yi, h->W, h->T, h->hcol, st);
    launch_add(m, h->hcol, d_dLdz, h->g, st);
    HIPCHK(h, hipMemsetAsync(h->flags + kCand + 2, 0, sizeof(int), st));
    launch_set_row(m, h->g, h->B + m, h->ldb, st);
    potrf_rows(h, m, m + 1, h->B, h->ldb, h->flags + kCand + 2);
    launch_potrs_bwd(m, h->B, h->ldb, h->B + m, h->ldb, d_gb, h->pflags_b, ++h->epoch, h->flags + kCand + 2, st);
    // dL/dA_0 = sym(X^ (sum_k lambda_k A_k - G_L) Y^{-1}) on E: the dX kernels with
    // M = G_L - sum_k lambda_k A_k, no beta mu term and a zero Xbar give -sym(X^ M Y^{-1})
    launch_assemble(d, d_gb, 0.0, 1.0, d_GL_E, h->G, st);
    launch_zcol(d, h->Xh, h->G, h->W, st);
    HIPCHK(h, hipMemsetAsync(h->Xn, 0, size_t(d.nslot) * sizeof(double), st));
    launch_dX_blocked(d, h->W, h->Yi, h->Xn, 0.0, h->part, d_gC_E, st);
    HIPCHK(h, hipGetLastError());
    h->metrics_ready = false;   // G was used as workspace: the next step recomputes it
    HIPCHK(h, hipStreamSynchronize(st));
    return check_flags(h, true);
}

sdpc_status sdpc_get_scm_timing(const sdpc_handle *h, double *ms5) {
    if (!h || !ms5) return SDPC_E_ARG;
    for (int i = 0; i < 5; ++i) ms5[i] = h->scm_ms[i];
    return SDPC_OK;
}

}  // extern "C"
