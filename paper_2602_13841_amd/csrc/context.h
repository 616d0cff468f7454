// Context and level data of the stmg library (internal).
#pragma once

#include "../../include/stmg.h"
#include "stmg_internal.h"

#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

namespace stmg {

// Serializes stream capture (V-cycle graphs) with the runtime calls that
// synchronize the whole device (allocation, free, stream destruction), which
// other host threads of the process (serving slots) may issue meanwhile.
inline std::recursive_mutex &device_api_mutex()
{
    static std::recursive_mutex m;
    return m;
}

struct HipError : std::runtime_error {
    int code;
    HipError(const std::string &m, int c) : std::runtime_error(m), code(c) {}
};

#define STMG_HIP(call)                                                                                       \
    do {                                                                                                     \
        hipError_t e_ = (call);                                                                              \
        if (e_ != hipSuccess)                                                                                \
            throw ::stmg::HipError(std::string(#call) + ": " + hipGetErrorString(e_), STMG_EHIP);           \
    } while (0)

// device allocation owned by a context
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    explicit DevBuf(size_t b) { alloc(b); }
    void alloc(size_t b)
    {
        release();
        if (b == 0) return;
        std::lock_guard<std::recursive_mutex> lk(device_api_mutex());
        if (hipMalloc(&p, b) != hipSuccess) {
            p = nullptr;
            throw HipError("device allocation of " + std::to_string(b) + " bytes failed", STMG_ENOMEM);
        }
        bytes = b;
    }
    void release()
    {
        if (p) {
            std::lock_guard<std::recursive_mutex> lk(device_api_mutex());
            (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
    }
    ~DevBuf() { release(); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes)
    {
        o.p = nullptr;
        o.bytes = 0;
    }
    DevBuf &operator=(DevBuf &&o) noexcept
    {
        if (this != &o) {
            release();
            p = o.p;
            bytes = o.bytes;
            o.p = nullptr;
            o.bytes = 0;
        }
        return *this;
    }
    template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

// Named device timers: hipEvent pairs recorded on the launching stream around
// kernels, accumulated per name when read back.  Off unless enabled.
struct Timers {
    bool on = false;
    struct Rec {
        std::string name;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<std::string, std::pair<double, long long>>> acc;
    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        STMG_HIP(hipEventCreate(&e));
        return e;
    }
    int begin(const char *name, hipStream_t s)
    {
        if (!on) return -1;
        Rec r{name, get(), get()};
        STMG_HIP(hipEventRecord(r.a, s));
        pending.push_back(r);
        return (int)pending.size() - 1;
    }
    void end(int idx, hipStream_t s)
    {
        if (idx >= 0) STMG_HIP(hipEventRecord(pending[idx].b, s));
    }
    void flush()
    {
        for (auto &r : pending) {
            STMG_HIP(hipEventSynchronize(r.b));
            float ms = 0;
            STMG_HIP(hipEventElapsedTime(&ms, r.a, r.b));
            bool found = false;
            for (auto &kv : acc)
                if (kv.first == r.name) {
                    kv.second.first += ms;
                    kv.second.second += 1;
                    found = true;
                }
            if (!found) acc.push_back({r.name, {double(ms), 1LL}});
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pending.clear();
    }
    ~Timers()
    {
        for (auto &r : pending) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

struct TimerScope {
    Timers *t;
    int idx;
    hipStream_t s;
    TimerScope(Timers *t_, const char *name, hipStream_t s_) : t(t_), idx(t_ ? t_->begin(name, s_) : -1), s(s_) {}
    ~TimerScope()
    {
        if (t && idx >= 0) t->end(idx, s);
    }
};

// one level of the hp hierarchy: (k, r) and a structured mesh
struct Level {
    int dim = 3, n[3] = {1, 1, 1}, r = 1, k = 0, nq = 4, npm = 1, nt = 1;
    unsigned dmask = 0;
    double nu = 1, tau = 1, g1 = 10, g2 = 10;
    bool mapped = false;
    long long ncell = 0, Nn = 0, Nv1 = 0, Np1 = 0, N = 0;
    int nl = 0;                      // (r+2)^d
    TimeCoefs tc{};
    TableLayout lay{};
    std::vector<double> vert_host;   // vertices (if mapped)
    DevBuf vert, tab64, tab32, E64, E32;
    DevBuf bcells;                   // cells with a face on the domain boundary
    int nbcell = 0;
    Timers *timers = nullptr;

    void init(const stmg_problem &p, int k_, int r_, int nx, int ny, int nz, int nq_,
              const std::vector<double> &verts);
    template <typename T> CellArgs<T> cell_args() const;
    template <typename T> GatherArgs<T> gather_args() const;
    // apply one of the cell operators (Jacobian, residual, mass) on stream s
    template <typename T>
    void apply(Mode mode, const T *state, const T *x, T *y, const T *rhs, const T *vprev, int nvec, hipStream_t s);
};

} // namespace stmg
