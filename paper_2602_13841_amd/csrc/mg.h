// hp space-time multigrid hierarchy, Krylov and Newton drivers (internal).
#pragma once

#include "context.h"
#include "transfers.h"
#include "vanka.h"
#include "vec_ops.h"

namespace stmg {

struct MgLevel {
    Level *L = nullptr;
    DevBuf st64, st32;            // level state (slab vector; velocity part used)
    DevBuf vstar;                 // midpoint velocity in the multigrid precision
    DevBuf elem;                  // element records
    DevBuf patches, piv, info;    // patch LU factors
    int m = 0;                    // patch size (full space-time patch)
    bool have_patches = false;
    // time-decoupled patches: one spatial factorization per eigen-system
    TimeDiag tdg{};
    int ms = 0;                   // spatial patch size
    long long sys_off[MAX_NT] = {0, 0, 0, 0}, piv_off[MAX_NT] = {0, 0, 0, 0};
    DevBuf perm;
    long long nfac = 0;           // factor entries of all systems (time-decoupled)
    DevBuf fac16;                 // BF16 copy of the FP32 factors (option)
    DevBuf dv_dinv, dv_schur, dv_piv;   // diagonal Vanka: D^{-1}, Schur LU, pivots
    DevBuf r, d, t, E;            // work vectors in the multigrid precision
};

// The FP64 preconditioner application (casts, V-cycle over all levels) as one
// captured HIP graph: replayed for every FGMRES iteration on fixed staging
// vectors; captured again after every rebuild or state change.
struct VcycleGraph {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    bool valid = false;    // captured for the current factors and states
    bool failed = false;   // capture not possible: eager V-cycles from then on
    bool warm = false;     // one eager V-cycle on the staging vectors has run
    DevBuf in, out;        // FP64 staging vectors of the captured cycle
    // private non-blocking stream the capture is recorded on (the caller's
    // stream may be the null stream, which cannot be captured, and other
    // threads' null-stream calls must not synchronize with a capture)
    hipStream_t cs = nullptr;
    void reset(hipStream_t s)
    {
        if (x || g) (void)hipStreamSynchronize(s);
        std::lock_guard<std::recursive_mutex> lk(device_api_mutex());
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
        x = nullptr;
        g = nullptr;
        valid = false;
    }
    ~VcycleGraph()
    {
        std::lock_guard<std::recursive_mutex> lk(device_api_mutex());
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
        if (cs) (void)hipStreamDestroy(cs);
    }
};

struct Mg {
    int prec = STMG_F32;
    double omega = 0.35;
    int weighting = 0;
    bool td = true;               // time-decoupled patch solves
    bool factor_bf16 = false;     // FP32 patch factors applied from a BF16 copy
    bool diag = false;            // diagonal Vanka (velocity blocks by their diagonal)
    bool diag_block = false;      // ... or by their node blocks (all components of a node)
    int nu1 = 1, nu2 = 1;
    std::vector<MgLevel> lv;
    std::vector<std::unique_ptr<Transfer>> tr;   // tr[l]: level l -> l+1
    // coarsest level direct solve (FP64)
    DevBuf cX, cY, cA, cpiv, cinfo, cr64, cx64;
    int cn = 0, cm = 0;
    bool border = false;
    bool state_set = false;
    size_t max_lds = 65536;
    bool use_graph = true;
    VcycleGraph graph;
};

// FGMRES and Newton workspace (FP64)
struct Krylov {
    int maxit = 0;
    long long N = 0;
    DevBuf V, MV, Z, w, u, h, partial, y;
    DevBuf H, cs, sn, g, report;            // Givens form of the Hessenberg system
    DevBuf r, Mr, dU, Ut, rt, tmp, dot;     // Newton vectors
    void ensure(long long N_, int maxit_);
};

void mg_build(stmg_ctx *ctx);
void mg_allocate(stmg_ctx *ctx);
void mg_set_state(stmg_ctx *ctx, const double *u);
void mg_rebuild(stmg_ctx *ctx);
// one Vanka sweep d <- d + omega S(r - J d); d_zero: d is known to be zero
// (first pre-smoothing step of a cycle), so the defect is r itself
template <typename T> void mg_smooth(stmg_ctx *ctx, int l, const T *r, T *d, bool d_zero = false);
template <typename T> void mg_vcycle(stmg_ctx *ctx, int l, const T *r, T *d);
// z = B v for FP64 vectors on the finest level (casts around the cycle)
void mg_precondition(stmg_ctx *ctx, const double *v, double *z);

struct FgmresOut {
    int its = 0;
    bool converged = false;
    std::vector<double> hist;
};
FgmresOut fgmres(stmg_ctx *ctx, const double *state, const double *b, double *x, double rtol, int maxit);
int newton_solve(stmg_ctx *ctx, double *u, stmg_stats *stats);

} // namespace stmg

struct stmg_ctx {
    // device memory of the context (declared first: released last, after
    // every buffer that points into it)
    stmg::Arena arena;
    stmg::DevBuf own_block;   // the arena's block when the library allocated it
    stmg_problem prob{};
    stmg_options opt{};
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<std::unique_ptr<stmg::Level>> levels;   // levels[0] = finest
    stmg::DevBuf rhs, vprev;                            // slab data (FP64)
    bool has_rhs = false, has_vprev = false;
    stmg::Timers timers;
    std::unique_ptr<stmg::Mg> mg;
    stmg::Krylov kry;
};
