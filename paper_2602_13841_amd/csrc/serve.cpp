// Serving loop for slab solves (continuous batching): requests of different
// mesh sizes and degrees arrive over time (host clock) and run concurrently,
// each in a slot = a host thread with its own HIP stream, so the kernels of
// admitted requests overlap on the device.  Each request's Newton/Krylov state
// stays on the device until it completes.
//
// Admission: when a slot is free, the earliest arrived request whose HBM
// footprint fits the budget is admitted (first fit in arrival order, so a
// large request waiting for memory does not block smaller ones behind it).
//
// Context pool: a finished request's context is kept, idle, under the key of
// its discretization (dimension, cells, degrees, geometry, boundary data,
// options); a later request with the same key takes it and only resets the
// viscosity and slab length (stmg_set_coefficients) instead of building the
// hierarchy, transfer matrices and workspace again.  Idle contexts count
// against the budget and are destroyed, oldest first, when an admission needs
// their memory.  Request vectors live in per-slot device buffers sized once for
// the largest request, so no device allocation happens per request once the
// pool is warm.
//
// Results do not depend on the mix: contexts share no device data, a reused
// context is reset before its next solve, and every kernel is deterministic.
#include "mg.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <list>
#include <mutex>
#include <thread>

using namespace stmg;

namespace {

double clock_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// requests that may share a context: everything but nu and tau
bool same_shape(const stmg_problem &a, const stmg_problem &b)
{
    if (a.dim != b.dim || a.r != b.r || a.k != b.k || a.dirichlet_faces != b.dirichlet_faces ||
        a.gamma1 != b.gamma1 || a.gamma2 != b.gamma2 || a.vertices != b.vertices)
        return false;
    for (int i = 0; i < a.dim; ++i)
        if (a.n_cells[i] != b.n_cells[i]) return false;
    return true;
}

struct Pooled {
    stmg_problem prob;
    stmg_ctx *ctx;
    size_t footprint;
};

} // namespace

extern "C" int stmg_serve(const stmg_request *reqs, int n, const stmg_options *opt, int slots, size_t hbm_budget,
                          stmg_request_result *res, double *wall_s)
{
    if (!reqs || n < 0 || !res || slots < 1) return STMG_EINVAL;
    stmg_options o;
    if (opt) o = *opt;
    else stmg_default_options(&o);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return STMG_EHIP;
    // without a budget: 85 % of the memory free at the start (bounds the pool)
    size_t budget = hbm_budget;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return STMG_EHIP;
        budget = (size_t)(0.85 * (double)fr);
    }
    std::vector<size_t> foot(n);
    long long maxN = 1;
    for (int i = 0; i < n; ++i) {
        foot[i] = stmg_footprint_bytes(&reqs[i].prob, &o);
        std::memset(&res[i], 0, sizeof(res[i]));
        res[i].footprint = foot[i];
        if (foot[i] == 0) return STMG_EINVAL;
        if (foot[i] > budget) return STMG_ENOMEM;
        const stmg_problem &p = reqs[i].prob;
        long long nn = 1, nc = 1;
        for (int a = 0; a < p.dim; ++a) {
            nn *= (long long)(p.r + 1) * p.n_cells[a] + 1;
            nc *= p.n_cells[a];
        }
        long long npm = 1;
        for (int j = 1; j <= p.dim; ++j) npm = npm * (p.r + j) / j;
        maxN = std::max(maxN, (long long)(p.k + 1) * (p.dim * nn + nc * npm));
    }
    // arrival order; a request leaves `waiting` when admitted
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return reqs[a].arrival_s < reqs[b].arrival_s; });
    std::list<int> waiting(order.begin(), order.end());
    std::list<Pooled> idle;                 // least recently used first
    std::mutex mu;
    std::condition_variable cv;
    size_t in_use = 0, idle_bytes = 0;     // footprints of running requests / idle contexts
    int done = 0;
    const char *ev = std::getenv("STMG_VERBOSE");
    const bool verbose = ev && *ev && *ev != '0';
    // per-slot request vectors (u, rhs, v_prev), sized for the largest request
    std::vector<double *> slot_buf(slots, nullptr);
    {
        std::lock_guard<std::recursive_mutex> lk(stmg::device_api_mutex());
        for (int sl = 0; sl < slots; ++sl)
            if (hipMalloc(&slot_buf[sl], (size_t)maxN * 8 * 3) != hipSuccess) {
                for (double *p : slot_buf)
                    if (p) (void)hipFree(p);
                return STMG_ENOMEM;
            }
    }
    const double t0 = clock_s();
    auto destroy = [](stmg_ctx *c) { stmg_destroy(c); };
    auto worker = [&](int slot) {
        (void)hipSetDevice(dev);
        // runtime calls of this thread stay legal while another slot records a
        // V-cycle graph on its own stream
        hipStreamCaptureMode mode = hipStreamCaptureModeRelaxed;
        (void)hipThreadExchangeStreamCaptureMode(&mode);
        hipStream_t s = nullptr;
        {
            std::lock_guard<std::recursive_mutex> lk(stmg::device_api_mutex());
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
        }
        double *du = slot_buf[slot], *drhs = du + maxN, *dvp = drhs + maxN;
        for (;;) {
            int idx = -1;
            stmg_ctx *ctx = nullptr;
            std::vector<stmg_ctx *> evict;
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    if (waiting.empty()) break;
                    const double now = clock_s() - t0;
                    double next_arrival = -1;
                    for (auto it = waiting.begin(); it != waiting.end(); ++it) {
                        const int cand = *it;
                        if (reqs[cand].arrival_s > now) {
                            next_arrival = reqs[cand].arrival_s;
                            break;                 // later ones have not arrived either
                        }
                        // a pooled context of the same shape is taken (its
                        // memory moves from idle to in use); a new context
                        // needs its footprint next to the running requests,
                        // idle contexts being evicted for it
                        auto hit = std::find_if(idle.begin(), idle.end(), [&](const Pooled &p) {
                            return same_shape(p.prob, reqs[cand].prob);
                        });
                        if (hit == idle.end() && in_use + foot[cand] > budget) continue;   // first fit
                        if (hit != idle.end()) {
                            ctx = hit->ctx;
                            foot[cand] = hit->footprint;
                            idle_bytes -= hit->footprint;
                            idle.erase(hit);
                        } else {
                            while (!idle.empty() && in_use + idle_bytes + foot[cand] > budget) {
                                evict.push_back(idle.front().ctx);
                                idle_bytes -= idle.front().footprint;
                                idle.pop_front();
                            }
                        }
                        in_use += foot[cand];
                        idx = cand;
                        waiting.erase(it);
                        break;
                    }
                    if (idx >= 0) break;
                    // nothing admissible: wait for the next arrival or a completion
                    if (next_arrival >= 0) cv.wait_for(lk, std::chrono::duration<double>(next_arrival - now));
                    else cv.wait(lk);
                }
            }
            for (stmg_ctx *c : evict) destroy(c);
            if (idx < 0) break;
            const stmg_request &q = reqs[idx];
            stmg_request_result &R = res[idx];
            R.start_s = clock_s() - t0;
            int rc = STMG_OK;
            R.reused_context = ctx ? 1 : 0;
            if (ctx) {
                // reused context: now on this slot's stream, with this request's coefficients
                ctx->stream = s;
                rc = stmg_set_coefficients(ctx, q.prob.nu, q.prob.tau);
            } else {
                rc = stmg_create(&q.prob, &o, nullptr, 0, s, &ctx);   // one allocation of its footprint
            }
            long long N = 0, Nv = 0;
            if (rc == STMG_OK) {
                stmg_sizes(ctx, &N, &Nv, nullptr);
                const long long Nv1 = Nv / (q.prob.k + 1);
                if (q.u_init) (void)hipMemcpyAsync(du, q.u_init, N * 8, hipMemcpyHostToDevice, s);
                else (void)vec_fill<double>(N, 0.0, du, s);
                if (q.rhs) (void)hipMemcpyAsync(drhs, q.rhs, N * 8, hipMemcpyHostToDevice, s);
                if (q.v_prev) (void)hipMemcpyAsync(dvp, q.v_prev, Nv1 * 8, hipMemcpyHostToDevice, s);
                rc = stmg_set_slab_data(ctx, q.rhs ? drhs : nullptr, q.v_prev ? dvp : nullptr);
                if (rc == STMG_OK) rc = stmg_newton_gmres_solve(ctx, du, &R.stats);
                if (rc >= 0 && q.u_out) (void)hipMemcpyAsync(q.u_out, du, N * 8, hipMemcpyDeviceToHost, s);
                (void)hipStreamSynchronize(s);
            }
            if (rc < 0) {
                std::fprintf(stderr, "[stmg] serve: request %d failed (%d): %s\n", idx, rc,
                             ctx ? stmg_last_error(ctx) : "context creation failed");
                std::fflush(stderr);
            }
            R.rc = rc;
            R.end_s = clock_s() - t0;
            R.latency_s = R.end_s - q.arrival_s;
            bool keep = ctx && rc >= 0;
            if (ctx && !keep) destroy(ctx);
            {
                std::lock_guard<std::mutex> lk(mu);
                in_use -= foot[idx];
                if (keep) {
                    idle.push_back(Pooled{q.prob, ctx, foot[idx]});
                    idle_bytes += foot[idx];
                }
                ++done;
                if (verbose) {
                    std::fprintf(stderr, "[stmg] serve %d/%d: request %d (%dD n=%d r=%d k=%d) rc %d, %.2f s in slot\n",
                                 done, n, idx, q.prob.dim, q.prob.n_cells[0], q.prob.r, q.prob.k, rc, R.end_s - R.start_s);
                    std::fflush(stderr);
                }
            }
            cv.notify_all();
        }
        std::lock_guard<std::recursive_mutex> lk(stmg::device_api_mutex());
        (void)hipStreamDestroy(s);
    };
    std::vector<std::thread> th;
    for (int i = 0; i < slots; ++i) th.emplace_back(worker, i);
    for (auto &t : th) t.join();
    for (auto &p : idle) destroy(p.ctx);
    {
        std::lock_guard<std::recursive_mutex> lk(stmg::device_api_mutex());
        for (double *p : slot_buf)
            if (p) (void)hipFree(p);
    }
    if (wall_s) *wall_s = clock_s() - t0;
    int worst = STMG_OK;
    for (int i = 0; i < n; ++i)
        if (res[i].rc < 0) worst = res[i].rc;
    return worst;
}
