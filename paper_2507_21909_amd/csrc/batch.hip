// Many (beta, h, D) instances of the RG flow in one call.
//
// Each instance is an independent solver state (its own arena, device state
// and HIP stream, default priority).  trg_batch_run drives them from a pool
// of host workers: a worker takes the next instance and runs all its steps,
// so the GPU holds several instances' kernels at once (one per worker stream)
// while each worker waits on its own instance's convergence read-backs.  Small
// D instances are latency-bound, and this overlap is where the throughput
// comes from.  The kernels are the single-instance kernels, so every instance
// gives bit for bit what a lone solver with the same options gives.
// trg_batch_run_graphs takes the host out of the steady part of each flow:
// once a step leaves an instance's shapes unchanged, one recorded step per
// axis (trg_graph_capture) is replayed for the rest of its steps, with one
// status read per step instead of one per Jacobi sweep; replays equal eager
// steps bit for bit.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "trg.h"

struct trg_batch {
    std::vector<trg_state *> s;
    std::vector<hipStream_t> streams;
    std::vector<double> beta, h;
    std::vector<int> D;
    int workers = 1;
    int device = 0;
    std::string err;
};

namespace {
constexpr int MAX_WORKERS = 8;

// Recording a step (trg_graph_capture) takes this lock exclusively and every
// other HIP-calling part of a worker's instance shares it, so no worker calls
// the runtime while another records (a precaution: a 128-instance run with
// graphs once stopped making progress, cause not identified).
std::shared_mutex hip_lock;

// all nsteps of one instance: eager steps, and with graphs, checked replays of
// recorded steps from the first step that leaves the shapes unchanged; a
// replay that fails is rolled back by the library and the step taken eagerly
// (an error there is the instance's error), then the steps are recorded again
int run_instance(trg_state *s, int nsteps, const int *axes, bool graphs) {
    trg_graph *g[4] = {nullptr, nullptr, nullptr, nullptr};
    auto drop = [&]() {
        for (trg_graph *&x : g) {
            trg_graph_destroy(x);
            x = nullptr;
        }
    };
    auto record = [&]() {
        std::unique_lock<std::shared_mutex> lk(hip_lock);
        int rc = TRG_OK;
        for (int a = 0; a < 4 && rc == TRG_OK; ++a) rc = trg_graph_capture(s, TRG_METHOD_TRIAD, a, &g[a]);
        if (rc != TRG_OK) drop();
        return rc;
    };
    auto shared = [&]() { return std::shared_lock<std::shared_mutex>(hip_lock); };
    static const bool trace = [] {
        const char *e = getenv("TRG_BATCH_TRACE");
        return e && *e && *e != '0';
    }();
    bool steady = false;
    int rc = TRG_OK, replays = 0, fallbacks = 0;
    for (int k = 0; k < nsteps && rc == TRG_OK; ++k) {
        const int ax = axes ? axes[k] : k % 4;
        if (steady) {
            {
                auto lk = shared();
                if (trg_graph_launch(g[ax], 1) == TRG_OK) {
                    ++replays;
                    continue;
                }
                ++fallbacks;
                drop();
                rc = triad_atrg_step(s, ax);
            }
            if (rc == TRG_OK && k + 1 < nsteps) rc = record();
            continue;
        }
        int d0[4], c0 = 0, d1[4], c1 = 0;
        if (graphs) rc = trg_shape(s, d0, &c0, nullptr);
        if (rc == TRG_OK) {
            auto lk = shared();
            rc = triad_atrg_step(s, ax);
        }
        if (rc == TRG_OK && graphs) {
            rc = trg_shape(s, d1, &c1, nullptr);
            if (rc == TRG_OK && c0 == c1 && std::equal(d0, d0 + 4, d1) && k + 1 < nsteps) {
                rc = record();
                steady = rc == TRG_OK;
            }
        }
    }
    {
        auto lk = shared();
        drop();
    }
    if (trace && graphs)
        fprintf(stderr, "[batch] %d replays, %d taken eagerly after a failed replay\n", replays, fallbacks);
    return rc;
}

int run_all(trg_batch *b, int nsteps, const int *axes, bool graphs) {
    if (!b || nsteps < 0) return TRG_E_INVALID;
    if (axes)
        for (int i = 0; i < nsteps; ++i)
            if (axes[i] < 0 || axes[i] > 3) return TRG_E_INVALID;
    const int n = (int)b->s.size();
    std::atomic<int> next{0};
    std::atomic<int> first_rc{TRG_OK};
    std::vector<std::string> errs(n);
    auto work = [&]() {
        (void)hipSetDevice(b->device);
        for (int i = next++; i < n; i = next++) {
            const int rc = run_instance(b->s[i], nsteps, axes, graphs);
            if (rc != TRG_OK) {
                errs[i] = trg_last_error(b->s[i]);
                int expect = TRG_OK;
                first_rc.compare_exchange_strong(expect, rc);
            }
            {   // bounded memory: one workspace per worker
                std::shared_lock<std::shared_mutex> lk(hip_lock);
                (void)trg_release_workspace(b->s[i]);
            }
        }
    };
    std::vector<std::thread> pool;
    for (int w = 1; w < b->workers; ++w) pool.emplace_back(work);
    work();
    for (auto &t : pool) t.join();
    b->err.clear();
    for (int i = 0; i < n; ++i)
        if (!errs[i].empty()) {
            b->err = "instance " + std::to_string(i) + ": " + errs[i];
            break;
        }
    return first_rc.load();
}
}  // namespace

extern "C" {

int trg_batch_create(int n, const double *betas, const double *hs, const int *Ds, const trg_options *opt,
                     trg_batch **out) {
    if (!out) return TRG_E_INVALID;
    *out = nullptr;
    if (n < 1 || !betas || !hs || !Ds || !opt || opt->stream) return TRG_E_INVALID;
    trg_batch *b = new (std::nothrow) trg_batch();
    if (!b) return TRG_E_NOMEM;
    b->device = opt->device;
    b->workers = std::min(n, MAX_WORKERS);
    if (hipSetDevice(opt->device) != hipSuccess) {
        delete b;
        return TRG_E_HIP;
    }
    for (int i = 0; i < n; ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            trg_batch_destroy(b);
            return TRG_E_HIP;
        }
        b->streams.push_back(st);
        trg_options o = *opt;
        o.stream = st;
        o.instance = opt->instance + (uint32_t)i;   // independent sketches per instance
        trg_state *s = nullptr;
        int rc = trg_create(&o, &s);
        if (rc == TRG_OK) {
            b->s.push_back(s);
            rc = tensor_init(s, TRG_MODEL_ISING, betas[i], hs[i], Ds[i]);
        }
        if (rc != TRG_OK) {
            trg_batch_destroy(b);
            return rc;
        }
        b->beta.push_back(betas[i]);
        b->h.push_back(hs[i]);
        b->D.push_back(Ds[i]);
    }
    *out = b;
    return TRG_OK;
}


int trg_batch_run(trg_batch *b, int nsteps, const int *axes) { return run_all(b, nsteps, axes, false); }

int trg_batch_run_graphs(trg_batch *b, int nsteps, const int *axes) { return run_all(b, nsteps, axes, true); }

int trg_batch_log_z(trg_batch *b, double *out_n) {
    if (!b || !out_n) return TRG_E_INVALID;
    for (size_t i = 0; i < b->s.size(); ++i) {
        const int rc = log_z_per_site(b->s[i], &out_n[i]);
        if (rc != TRG_OK) {
            b->err = "instance " + std::to_string(i) + ": " + trg_last_error(b->s[i]);
            return rc;
        }
    }
    return TRG_OK;
}

int trg_batch_size(const trg_batch *b) { return b ? (int)b->s.size() : 0; }

const char *trg_batch_last_error(const trg_batch *b) { return b ? b->err.c_str() : ""; }

int trg_batch_destroy(trg_batch *b) {
    if (!b) return TRG_OK;
    for (trg_state *s : b->s) trg_destroy(s);
    (void)hipSetDevice(b->device);
    for (hipStream_t st : b->streams) (void)hipStreamDestroy(st);
    delete b;
    return TRG_OK;
}

}  // extern "C"
