// sdpc_batch_solve: many independent SDPs of uneven sizes on one GPU.
//
// One instance alone leaves most of the chip idle: its sparse factorisations and
// substitutions are chains of block steps run by one wave or one workgroup, and
// every iteration waits for its host-side stopping test.  The batch keeps many
// instances in flight instead, each on the stream of a host worker:
//   1. analysis   the host symbolic phase of every instance (sdpc_analyze),
//                 spread over the workers;
//   2. tuning     per size class (largest clique x order), the storage-block
//                 width of the clique tiles is chosen by timing real iterations
//                 of the class's largest instance at a few widths;
//   3. placement  longest estimated work first onto the least loaded worker;
//   4. create     every handle is created up front: device memory is allocated
//                 before any solve starts (288 GB of HBM hold the whole batch),
//                 so no allocation or release interrupts the solves;
//   5. solve      each worker runs its instances' iterations back to back on its
//                 own stream; an instance retires as soon as its stopping test
//                 holds, and the worker moves on to its next one;
//   6. release    after every worker has finished.
// The Schur complement phase, the dense Cholesky and the loop closure of each
// instance are the library's own (sdpc_solve), so every instance's arithmetic
// is that of the plain solver with the chosen block width.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/sdpc.h"
#include "kernels.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// Runs f(i) for i in [0, count) on `workers` host threads.
void parallel_for(int count, int workers, const std::function<void(int)> &f) {
    std::atomic<int> next(0);
    std::vector<std::thread> th;
    for (int w = 0; w < std::max(1, std::min(workers, count)); ++w)
        th.emplace_back([&] {
            for (int i = next++; i < count; i = next++) f(i);
        });
    for (auto &t : th) t.join();
}

class Barrier {
public:
    explicit Barrier(int n) : n_(n) {}
    void wait() {
        std::unique_lock<std::mutex> lk(mu_);
        const int gen = gen_;
        if (++count_ == n_) {
            count_ = 0;
            ++gen_;
            cv_.notify_all();
        } else {
            cv_.wait(lk, [&] { return gen != gen_; });
        }
    }

private:
    std::mutex mu_;
    std::condition_variable cv_;
    int n_, count_ = 0, gen_ = 0;
};

// size class: largest clique (<= 8, <= 16, more) x order (<= 200, <= 500, more)
int size_class(const sdpc_analysis &a, int n) {
    const int c = a.max_clique <= 8 ? 0 : (a.max_clique <= 16 ? 1 : 2);
    const int s = n <= 200 ? 0 : (n <= 500 ? 1 : 2);
    return 3 * c + s;
}

// work estimate: the dense SCM Cholesky plus the latency of the block walks
double work_estimate(const sdpc_analysis &a, int m) {
    return double(m) * m * m / 3.0 + 2.0e5 * a.nblocks;
}

constexpr int kTuneWidths[] = {8, 16, 32};

}  // namespace

extern "C" {

sdpc_batch_options sdpc_default_batch_options(void) {
    sdpc_batch_options o;
    std::memset(&o, 0, sizeof(o));
    o.workers = 8;
    o.autotune = 1;
    o.dual_points = 32;
    return o;
}

sdpc_status sdpc_batch_solve(int32_t count, const sdpc_problem *probs, const sdpc_params *params,
                             sdpc_batch_options *opt, sdpc_result *results, double *const *d_z) {
    using sdpc::set_unbound_error;
    if (count < 0 || (count > 0 && (!probs || !results))) {
        set_unbound_error("sdpc_batch_solve: bad arguments");
        return SDPC_E_ARG;
    }
    sdpc_batch_options o = opt ? *opt : sdpc_default_batch_options();
    if (o.workers < 1 || o.workers > 64) {
        set_unbound_error("sdpc_batch_solve: workers must be 1..64");
        return SDPC_E_ARG;
    }
    const auto t_all = Clock::now();
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_unbound_error("sdpc_batch_solve: no current device");
        return SDPC_E_HIP;
    }
    for (int i = 0; i < count; ++i) std::memset(&results[i], 0, sizeof(sdpc_result));
    auto prm_of = [&](int i) {
        sdpc_params p = params ? params[i] : sdpc_default_params();
        if (p.dual_points == 0) p.dual_points = o.dual_points;
        return p;
    };
    // ---- 1. analysis
    std::vector<sdpc_analysis> info(count);
    std::vector<int> ok(count, 0);
    parallel_for(count, o.workers, [&](int i) {
        const sdpc_params p = prm_of(i);
        const sdpc_status s = sdpc_analyze(&probs[i], &p, &info[i], nullptr, nullptr, nullptr, nullptr);
        results[i].status = s;
        ok[i] = (s == SDPC_OK);
    });
    // ---- 2. tuning of the block width per size class
    const auto t_tune = Clock::now();
    int width[9];
    for (int c = 0; c < 9; ++c) width[c] = 0;   // 0: the instance's own block_width
    if (o.autotune) {
        std::vector<int> rep(9, -1);
        for (int i = 0; i < count; ++i) {
            if (!ok[i]) continue;
            const int c = size_class(info[i], probs[i].n);
            if (rep[c] < 0 || work_estimate(info[i], probs[i].m) > work_estimate(info[rep[c]], probs[rep[c]].m))
                rep[c] = i;
        }
        std::vector<int> classes;
        for (int c = 0; c < 9; ++c)
            if (rep[c] >= 0) classes.push_back(c);
        parallel_for(int(classes.size()), o.workers, [&](int t) {
            const int c = classes[t], i = rep[c];
            (void)hipSetDevice(dev);
            hipStream_t st = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
            double best = 1e300;
            for (int bw : kTuneWidths) {
                sdpc_params p = prm_of(i);
                p.block_width = bw;
                sdpc_handle *h = nullptr;
                if (sdpc_create(&probs[i], &p, st, &h) != SDPC_OK) continue;
                sdpc_result r;
                // the first step pays for the cold start; the next two are timed
                bool good = sdpc_step(h, &r) == SDPC_OK;
                const auto t0 = Clock::now();
                for (int k = 0; k < 2 && good; ++k) good = sdpc_step(h, &r) == SDPC_OK;
                const double ms = ms_since(t0);
                sdpc_destroy(h);
                if (good && ms < best) {
                    best = ms;
                    width[c] = bw;
                }
            }
            (void)hipStreamDestroy(st);
        });
    }
    o.tune_ms = ms_since(t_tune);
    for (int c = 0; c < 9; ++c) o.tuned_width[c] = width[c];
    // ---- 3. placement: longest work first onto the least loaded worker
    const int W = std::max(1, std::min<int>(o.workers, count));
    std::vector<int> order;
    for (int i = 0; i < count; ++i)
        if (ok[i]) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return work_estimate(info[a], probs[a].m) > work_estimate(info[b], probs[b].m);
    });
    std::vector<std::vector<int>> mine(W);
    std::vector<double> load(W, 0.0);
    for (int i : order) {
        const int w = int(std::min_element(load.begin(), load.end()) - load.begin());
        mine[w].push_back(i);
        load[w] += work_estimate(info[i], probs[i].m);
    }
    // ---- 4-6. create everything, solve, release
    std::vector<sdpc_handle *> hs(count, nullptr);
    Barrier bar(W);
    std::vector<double> t_create(W, 0.0), t_solve(W, 0.0);
    std::vector<std::thread> th;
    for (int w = 0; w < W; ++w)
        th.emplace_back([&, w] {
            (void)hipSetDevice(dev);
            hipStream_t st = nullptr;
            const bool have_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
            auto t0 = Clock::now();
            for (int i : mine[w]) {
                if (!have_stream) {
                    results[i].status = SDPC_E_HIP;
                    continue;
                }
                sdpc_params p = prm_of(i);
                const int bw = width[size_class(info[i], probs[i].n)];
                if (bw > 0) p.block_width = bw;
                const sdpc_status s = sdpc_create(&probs[i], &p, st, &hs[i]);
                if (s != SDPC_OK) {
                    results[i].status = s;
                    hs[i] = nullptr;
                }
            }
            t_create[w] = ms_since(t0);
            bar.wait();   // no allocation while any instance is being solved
            t0 = Clock::now();
            for (int i : mine[w]) {
                if (!hs[i]) continue;
                sdpc_solve(hs[i], &results[i]);
                if (d_z && d_z[i]) sdpc_get_solution(hs[i], nullptr, nullptr, d_z[i]);
            }
            t_solve[w] = ms_since(t0);
            bar.wait();
            for (int i : mine[w])
                if (hs[i]) sdpc_destroy(hs[i]);
            if (have_stream) (void)hipStreamDestroy(st);
        });
    for (auto &t : th) t.join();
    o.create_ms = *std::max_element(t_create.begin(), t_create.end());
    o.solve_ms = *std::max_element(t_solve.begin(), t_solve.end());
    o.total_ms = ms_since(t_all);
    if (opt) *opt = o;
    for (int i = 0; i < count; ++i)
        if (results[i].status != SDPC_OK) {
            set_unbound_error("sdpc_batch_solve: instance " + std::to_string(i) + " ended with status " +
                              std::to_string(results[i].status));
            return sdpc_status(results[i].status);
        }
    return SDPC_OK;
}

}  // extern "C"
