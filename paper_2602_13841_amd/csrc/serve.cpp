// Serving loop for slab solves: requests of different mesh sizes and degrees
// arrive over time (host clock), are admitted while a slot and the HBM
// budget allow (FIFO, admission by the footprint of the request), and run
// concurrently: every slot is a host thread with its own HIP stream and
// context, so the kernels of admitted requests overlap on the device.  Each
// request's Newton/Krylov state stays on the device until it completes.
// Results do not depend on the mix: contexts share no device data and every
// kernel is deterministic.
#include "mg.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <thread>

using namespace stmg;

namespace {

double clock_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

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
    std::vector<size_t> foot(n);
    for (int i = 0; i < n; ++i) {
        foot[i] = stmg_footprint_bytes(&reqs[i].prob, &o);
        std::memset(&res[i], 0, sizeof(res[i]));
        res[i].footprint = foot[i];
        if (foot[i] == 0) return STMG_EINVAL;
        if (hbm_budget && foot[i] > hbm_budget) return STMG_ENOMEM;
    }
    // FIFO by arrival time
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return reqs[a].arrival_s < reqs[b].arrival_s; });
    std::mutex mu;
    std::condition_variable cv;
    size_t in_use = 0;
    int next = 0, done = 0;
    // progress log on stderr when the environment variable STMG_VERBOSE is set
    const char *ev = std::getenv("STMG_VERBOSE");
    const bool verbose = ev && *ev && *ev != '0';
    const double t0 = clock_s();
    auto worker = [&]() {
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
        for (;;) {
            int idx = -1;
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    if (next >= n) break;
                    int cand = order[next];
                    double now = clock_s() - t0;
                    bool arrived = reqs[cand].arrival_s <= now;
                    bool fits = hbm_budget == 0 || in_use + foot[cand] <= hbm_budget;
                    if (arrived && fits) {
                        idx = cand;
                        in_use += foot[cand];
                        ++next;
                        break;
                    }
                    if (!arrived)
                        cv.wait_for(lk, std::chrono::duration<double>(reqs[cand].arrival_s - now));
                    else
                        cv.wait(lk);
                }
            }
            if (idx < 0) break;
            const stmg_request &q = reqs[idx];
            stmg_request_result &R = res[idx];
            R.start_s = clock_s() - t0;
            stmg_ctx *ctx = nullptr;
            int rc = stmg_create(&q.prob, &o, s, &ctx);
            double *du = nullptr, *drhs = nullptr, *dvp = nullptr;
            long long N = 0, Nv = 0;
            if (rc == STMG_OK) {
                stmg_sizes(ctx, &N, &Nv, nullptr);
                long long Nv1 = Nv / (q.prob.k + 1);
                bool ok;
                {
                    std::lock_guard<std::recursive_mutex> lk(stmg::device_api_mutex());
                    ok = hipMalloc(&du, N * 8) == hipSuccess;
                    if (ok && q.rhs) ok = hipMalloc(&drhs, N * 8) == hipSuccess;
                    if (ok && q.v_prev) ok = hipMalloc(&dvp, Nv1 * 8) == hipSuccess;
                }
                if (!ok) rc = STMG_ENOMEM;
                if (rc == STMG_OK) {
                    if (q.u_init) (void)hipMemcpyAsync(du, q.u_init, N * 8, hipMemcpyHostToDevice, s);
                    else (void)hipMemsetAsync(du, 0, N * 8, s);
                    if (drhs) (void)hipMemcpyAsync(drhs, q.rhs, N * 8, hipMemcpyHostToDevice, s);
                    if (dvp) (void)hipMemcpyAsync(dvp, q.v_prev, Nv1 * 8, hipMemcpyHostToDevice, s);
                    rc = stmg_set_slab_data(ctx, drhs, dvp);
                    if (rc == STMG_OK) rc = stmg_newton_gmres_solve(ctx, du, &R.stats);
                    if (rc >= 0 && q.u_out) {
                        (void)hipMemcpyAsync(q.u_out, du, N * 8, hipMemcpyDeviceToHost, s);
                        (void)hipStreamSynchronize(s);
                    }
                }
            }
            {
                std::lock_guard<std::recursive_mutex> lk(stmg::device_api_mutex());
                if (du) (void)hipFree(du);
                if (drhs) (void)hipFree(drhs);
                if (dvp) (void)hipFree(dvp);
            }
            if (rc < 0) {
                std::fprintf(stderr, "[stmg] serve: request %d failed (%d): %s\n", idx, rc,
                             ctx ? stmg_last_error(ctx) : "context creation failed");
                std::fflush(stderr);
            }
            if (ctx) stmg_destroy(ctx);
            (void)hipStreamSynchronize(s);
            R.rc = rc;
            R.end_s = clock_s() - t0;
            R.latency_s = R.end_s - q.arrival_s;
            {
                std::lock_guard<std::mutex> lk(mu);
                in_use -= foot[idx];
                if (verbose) {
                    ++done;
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
    for (int i = 0; i < slots; ++i) th.emplace_back(worker);
    for (auto &t : th) t.join();
    if (wall_s) *wall_s = clock_s() - t0;
    int worst = STMG_OK;
    for (int i = 0; i < n; ++i)
        if (res[i].rc < 0) worst = res[i].rc;
    return worst;
}
