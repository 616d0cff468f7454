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

// The device memory of one context: one block (the caller's workspace, or a
// single library allocation) handed out in creation order, each piece on a
// 256-byte boundary.  In counting mode no memory exists: only the sizes are
// added up (this is how stmg_footprint_bytes measures a context, by running
// the same construction code), and no device work may be issued.
struct Arena {
    unsigned char *base = nullptr;
    size_t cap = 0, used = 0;
    bool counting = false;
    static constexpr size_t ALIGN = 256;
    void *take(size_t b)
    {
        const size_t off = (used + ALIGN - 1) & ~(ALIGN - 1);
        if (!counting && off + b > cap)
            throw HipError("context workspace exhausted: " + std::to_string(off + b) + " of " +
                               std::to_string(cap) + " bytes", STMG_ENOMEM);
        used = off + b;
        // counting mode: a distinct non-null address that is never dereferenced
        return counting ? reinterpret_cast<void *>(ALIGN + off) : base + off;
    }
};

// arena that DevBuf allocations of the calling thread draw from (null: none)
inline Arena *&current_arena()
{
    static thread_local Arena *a = nullptr;
    return a;
}

struct ArenaScope {
    Arena *prev;
    explicit ArenaScope(Arena *a) : prev(current_arena()) { current_arena() = a; }
    ~ArenaScope() { current_arena() = prev; }
};

// true while a context is being measured (no device work allowed)
inline bool arena_counting()
{
    return current_arena() && current_arena()->counting;
}

// device buffer of a context: a piece of the current arena when one is set
// (released with the arena), else its own allocation
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool from_arena = false;
    DevBuf() = default;
    explicit DevBuf(size_t b) { alloc(b); }
    void alloc(size_t b)
    {
        release();
        if (b == 0) return;
        if (Arena *a = current_arena()) {
            p = a->take(b);
            bytes = b;
            from_arena = true;
            return;
        }
        std::lock_guard<std::recursive_mutex> lk(device_api_mutex());
        if (hipMalloc(&p, b) != hipSuccess) {
            p = nullptr;
            throw HipError("device allocation of " + std::to_string(b) + " bytes failed", STMG_ENOMEM);
        }
        bytes = b;
    }
    // a buffer of at least b bytes must exist (allocated when the context was built)
    void require(size_t b, const char *what) const
    {
        if (bytes < b)
            throw HipError(std::string("workspace buffer ") + what + " smaller than needed", STMG_ESTATE);
    }
    void release()
    {
        if (p && !from_arena) {
            std::lock_guard<std::recursive_mutex> lk(device_api_mutex());
            (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
        from_arena = false;
    }
    ~DevBuf() { release(); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), from_arena(o.from_arena)
    {
        o.p = nullptr;
        o.bytes = 0;
        o.from_arena = false;
    }
    DevBuf &operator=(DevBuf &&o) noexcept
    {
        if (this != &o) {
            release();
            p = o.p;
            bytes = o.bytes;
            from_arena = o.from_arena;
            o.p = nullptr;
            o.bytes = 0;
            o.from_arena = false;
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

    int nvec_cap64 = 1, nvec_cap32 = 1;   // vectors one operator launch handles (work buffer size)

    void init(const stmg_problem &p, int k_, int r_, int nx, int ny, int nz, int nq_,
              const std::vector<double> &verts);
    // cell-local result buffers for nvec64 FP64 and nvec32 FP32 vectors per
    // launch (0: that precision not used on this level)
    void alloc_work(int nvec64, int nvec32);
    template <typename T> CellArgs<T> cell_args() const;
    template <typename T> GatherArgs<T> gather_args() const;
    // apply one of the cell operators (Jacobian, residual, mass) on stream s
    template <typename T>
    void apply(Mode mode, const T *state, const T *x, T *y, const T *rhs, const T *vprev, int nvec, hipStream_t s);
};

} // namespace stmg
