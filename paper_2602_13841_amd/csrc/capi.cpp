// extern "C" entry points of the stmg library.
#include "lu_batch.h"
#include "lu_tuning.h"
#include "mg.h"

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

using namespace stmg;

namespace {

int fail(stmg_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

template <typename F> int guarded(stmg_ctx *ctx, F &&f)
{
    try {
        return f();
    } catch (const HipError &e) {
        return fail(ctx, e.code, e.what());
    } catch (const std::exception &e) {
        return fail(ctx, STMG_EINVAL, e.what());
    }
}

bool check_problem(const stmg_problem *p, std::string &why)
{
    if (!p) { why = "problem is NULL"; return false; }
    if (p->dim != 2 && p->dim != 3) { why = "dim must be 2 or 3"; return false; }
    for (int a = 0; a < p->dim; ++a)
        if (p->n_cells[a] < 1) { why = "n_cells must be >= 1"; return false; }
    if (p->r < 1 || p->r > 3) { why = "r must be in 1..3"; return false; }
    if (p->k < 0 || p->k > MAX_K) { why = "k must be in 0..3"; return false; }
    if (!(p->tau > 0) || !(p->nu > 0)) { why = "tau and nu must be positive"; return false; }
    // transfer matrices and node gathers index the velocity nodes of one
    // component with 32 bits; a p-transfer row holds up to 3^d entries
    long long nodes = 1;
    for (int a = 0; a < p->dim; ++a) nodes *= (long long)(p->r + 1) * p->n_cells[a] + 1;
    if (nodes > INT_MAX / 27) { why = "mesh too large (velocity nodes per component above 2^31 / 27)"; return false; }
    return true;
}

// enumerated and counted options outside their documented ranges are
// rejected rather than read as the nearest meaning
bool check_options(const stmg_options *o, std::string &why)
{
    if (!o) return true;
    auto flag = [](int v) { return v == 0 || v == 1; };
    if (o->prec_mg != STMG_F64 && o->prec_mg != STMG_F32) { why = "prec_mg must be STMG_F64 or STMG_F32"; return false; }
    if (o->n_q < 0 || o->max_levels < 0 || o->nu1 < 0 || o->nu2 < 0) {
        why = "n_q, max_levels, nu1 and nu2 must be >= 0";
        return false;
    }
    if (o->newton_maxit < 1 || o->fgmres_maxit < 1) { why = "newton_maxit and fgmres_maxit must be >= 1"; return false; }
    if (!(o->vanka_omega >= 0) || !(o->newton_rtol >= 0) || !(o->newton_atol >= 0)) {
        why = "vanka_omega, newton_rtol and newton_atol must be >= 0";
        return false;
    }
    if (!flag(o->vanka_weighting) || !flag(o->vanka_time_decoupled) || !flag(o->use_graphs) ||
        !flag(o->time_coarsening) || !flag(o->vanka_factor_bf16)) {
        why = "vanka_weighting, vanka_time_decoupled, use_graphs, time_coarsening and vanka_factor_bf16 must be 0 or 1";
        return false;
    }
    if (o->vanka_diagonal < 0 || o->vanka_diagonal > 2) { why = "vanka_diagonal must be 0, 1 or 2"; return false; }
    return true;
}

} // namespace

extern "C" {

void stmg_default_options(stmg_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->n_q = 0;
    o->max_levels = 0;
    o->nu1 = 1;
    o->nu2 = 1;
    o->vanka_omega = 0.0;
    o->prec_mg = STMG_F32;
    o->newton_rtol = 1e-8;
    o->newton_atol = 1e-12;
    o->newton_maxit = 30;
    o->ew_eta0 = 0.4;
    o->ew_c = 0.5;
    o->ew_theta = 1.5;
    o->ew_eta_min = 1e-3;
    o->ew_eta_max = 0.8;
    o->ls_lambda0 = 1.0;
    o->ls_c = 1e-4;
    o->ls_tau = 0.5;
    o->ls_alpha_min = 1e-3;
    o->ls_window = 5;
    o->ls_max_backtracks = 5;
    o->rb_theta_N = 0.5;
    o->rb_theta_L = 2.0;
    o->rb_kappa_abs = 10.0;
    o->rb_stag_theta = 0.9;
    o->rb_stag_s = 3;
    o->fgmres_maxit = 50;
    o->vanka_weighting = 1;
    o->vanka_time_decoupled = 1;
    o->use_graphs = 1;
    o->time_coarsening = 0;
    o->vanka_factor_bf16 = 0;
    o->vanka_diagonal = 0;
}

namespace {

// Builds the levels, transfers and every buffer of a context, all drawn from
// ctx->arena (counting mode: sizes only, no device work).
void build_context(stmg_ctx *ctx, const stmg_problem *prob)
{
    ArenaScope scope(&ctx->arena);
    std::vector<double> verts;
    if (prob->vertices) {
        long long nv = 1;
        for (int a = 0; a < prob->dim; ++a) nv *= prob->n_cells[a] + 1;
        verts.assign(prob->vertices, prob->vertices + nv * prob->dim);
    }
    auto L = std::make_unique<Level>();
    L->init(*prob, prob->k, prob->r, prob->n_cells[0], prob->n_cells[1], prob->dim == 3 ? prob->n_cells[2] : 1,
            ctx->opt.n_q, verts);
    if (L->nq != default_nq(L->r) && L->nq != L->r + 2) throw std::runtime_error("n_q must be ceil((3r+4)/2) or r+2");
    L->timers = &ctx->timers;
    ctx->levels.push_back(std::move(L));
    mg_build(ctx);
}

stmg_ctx *new_context(const stmg_problem *prob, const stmg_options *opt, void *stream)
{
    stmg_ctx *ctx = new stmg_ctx();
    ctx->prob = *prob;
    ctx->prob.vertices = nullptr;
    if (opt) ctx->opt = *opt;
    else stmg_default_options(&ctx->opt);
    ctx->stream = (hipStream_t)stream;
    return ctx;
}

// bytes a context of this problem consumes: the construction run in counting
// mode (0 if it cannot be built)
size_t measure_context(const stmg_problem *prob, const stmg_options *opt)
{
    std::unique_ptr<stmg_ctx> ctx(new_context(prob, opt, nullptr));
    ctx->arena.counting = true;
    try {
        build_context(ctx.get(), prob);
    } catch (const std::exception &) {
        return 0;
    }
    return (ctx->arena.used + Arena::ALIGN - 1) & ~(Arena::ALIGN - 1);
}

void verbose_reject(const char *what, const std::string &why)
{
    const char *ev = std::getenv("STMG_VERBOSE");
    if (ev && *ev && *ev != '0') {
        std::fprintf(stderr, "[stmg] %s: %s\n", what, why.c_str());
        std::fflush(stderr);
    }
}

} // namespace

int stmg_create(const stmg_problem *prob, const stmg_options *opt, void *workspace, size_t ws_bytes, void *stream,
                stmg_ctx **out)
{
    if (!out) return STMG_EINVAL;
    *out = nullptr;
    std::string why;
    if (!check_problem(prob, why) || !check_options(opt, why)) {
        verbose_reject("create rejected", why);
        return STMG_EINVAL;
    }
    const size_t need = measure_context(prob, opt);
    if (need == 0) {
        verbose_reject("create rejected", "the problem cannot be laid out");
        return STMG_EINVAL;
    }
    if (workspace && ((uintptr_t)workspace % Arena::ALIGN != 0)) {
        verbose_reject("create rejected", "workspace not aligned to 256 bytes");
        return STMG_EINVAL;
    }
    if (workspace && ws_bytes < need) {
        verbose_reject("create rejected", "workspace of " + std::to_string(ws_bytes) + " bytes, " +
                                              std::to_string(need) + " needed");
        return STMG_ENOMEM;
    }
    stmg_ctx *ctx = new_context(prob, opt, stream);
    int rc = guarded(ctx, [&]() {
        // construction issues synchronous copies: never concurrent with another
        // thread's V-cycle capture
        std::lock_guard<std::recursive_mutex> lk(device_api_mutex());
        if (workspace) {
            ctx->arena.base = static_cast<unsigned char *>(workspace);
            ctx->arena.cap = ws_bytes;
        } else {
            ctx->own_block.alloc(need);   // the one device allocation of the context
            ctx->arena.base = ctx->own_block.as<unsigned char>();
            ctx->arena.cap = need;
        }
        build_context(ctx, prob);
        return STMG_OK;
    });
    if (rc != STMG_OK) {
        verbose_reject("create failed", std::to_string(rc) + " " + ctx->err);
        delete ctx;
        return rc;
    }
    *out = ctx;
    return STMG_OK;
}

size_t stmg_workspace_used(const stmg_ctx *ctx) { return ctx ? ctx->arena.used : 0; }

int stmg_destroy(stmg_ctx *ctx)
{
    std::lock_guard<std::recursive_mutex> lk(device_api_mutex());
    delete ctx;
    return STMG_OK;
}

const char *stmg_last_error(const stmg_ctx *ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

size_t stmg_footprint_bytes(const stmg_problem *prob, const stmg_options *opt)
{
    std::string why;
    if (!check_problem(prob, why) || !check_options(opt, why)) return 0;
    return measure_context(prob, opt);
}

int stmg_set_coefficients(stmg_ctx *ctx, double nu, double tau)
{
    if (!ctx || !(nu > 0) || !(tau > 0)) return fail(ctx, STMG_EINVAL, "nu and tau must be positive");
    return guarded(ctx, [&]() {
        STMG_HIP(hipStreamSynchronize(ctx->stream));
        for (auto &L : ctx->levels) {
            L->nu = nu;
            L->tau = tau;
            L->tc = time_coefficients(L->k, tau);
        }
        ctx->prob.nu = nu;
        ctx->prob.tau = tau;
        Mg &mg = *ctx->mg;
        mg.graph.reset(ctx->stream);
        mg.state_set = false;
        for (auto &M : mg.lv) M.have_patches = false;
        return STMG_OK;
    });
}

int stmg_sizes(const stmg_ctx *ctx, long long *n_total, long long *n_velocity, long long *n_pressure)
{
    if (!ctx || ctx->levels.empty()) return STMG_EINVAL;
    const Level &L = *ctx->levels[0];
    if (n_total) *n_total = L.N;
    if (n_velocity) *n_velocity = L.nt * L.Nv1;
    if (n_pressure) *n_pressure = L.nt * L.Np1;
    return STMG_OK;
}

int stmg_set_slab_data(stmg_ctx *ctx, const double *rhs, const double *v_prev)
{
    if (!ctx) return STMG_EINVAL;
    return guarded(ctx, [&]() {
        const Level &L = *ctx->levels[0];
        if (rhs) {
            ctx->rhs.require((size_t)L.N * 8, "rhs");
            STMG_HIP(hipMemcpyAsync(ctx->rhs.p, rhs, (size_t)L.N * 8, hipMemcpyDeviceToDevice, ctx->stream));
        }
        ctx->has_rhs = rhs != nullptr;
        if (v_prev) {
            ctx->vprev.require((size_t)L.Nv1 * 8, "v_prev");
            STMG_HIP(hipMemcpyAsync(ctx->vprev.p, v_prev, (size_t)L.Nv1 * 8, hipMemcpyDeviceToDevice, ctx->stream));
        }
        ctx->has_vprev = v_prev != nullptr;
        return STMG_OK;
    });
}

int stmg_residual(stmg_ctx *ctx, const double *u, double *r)
{
    if (!ctx || !u || !r) return fail(ctx, STMG_EINVAL, "NULL argument");
    return guarded(ctx, [&]() {
        Level &L = *ctx->levels[0];
        L.apply<double>(Mode::Res, nullptr, u, r, ctx->has_rhs ? ctx->rhs.as<double>() : nullptr,
                        ctx->has_vprev ? ctx->vprev.as<double>() : nullptr, 1, ctx->stream);
        return STMG_OK;
    });
}

int stmg_jacobian_vmult_batched(stmg_ctx *ctx, int prec, const void *u_state, const void *x, void *y, int nvec)
{
    if (!ctx || !u_state || !x || !y || nvec < 1) return fail(ctx, STMG_EINVAL, "invalid argument");
    return guarded(ctx, [&]() {
        Level &L = *ctx->levels[0];
        if (prec == STMG_F64)
            L.apply<double>(Mode::Jac, (const double *)u_state, (const double *)x, (double *)y, nullptr, nullptr, nvec,
                            ctx->stream);
        else if (prec == STMG_F32)
            L.apply<float>(Mode::Jac, (const float *)u_state, (const float *)x, (float *)y, nullptr, nullptr, nvec,
                           ctx->stream);
        else
            return fail(ctx, STMG_EINVAL, "prec must be STMG_F64 or STMG_F32");
        return STMG_OK;
    });
}

int stmg_jacobian_vmult(stmg_ctx *ctx, int prec, const void *u_state, const void *x, void *y)
{
    return stmg_jacobian_vmult_batched(ctx, prec, u_state, x, y, 1);
}

int stmg_mass_vmult(stmg_ctx *ctx, int prec, const void *x, void *y)
{
    if (!ctx || !x || !y) return fail(ctx, STMG_EINVAL, "NULL argument");
    return guarded(ctx, [&]() {
        Level &L = *ctx->levels[0];
        if (prec == STMG_F64)
            L.apply<double>(Mode::Mass, nullptr, (const double *)x, (double *)y, nullptr, nullptr, 1, ctx->stream);
        else if (prec == STMG_F32)
            L.apply<float>(Mode::Mass, nullptr, (const float *)x, (float *)y, nullptr, nullptr, 1, ctx->stream);
        else
            return fail(ctx, STMG_EINVAL, "prec must be STMG_F64 or STMG_F32");
        return STMG_OK;
    });
}

int stmg_num_levels(const stmg_ctx *ctx)
{
    return ctx ? (int)ctx->levels.size() : STMG_EINVAL;
}

int stmg_level_info(const stmg_ctx *ctx, int level, int *k, int *r, int *n_cells, long long *n_total)
{
    if (!ctx || level < 0 || level >= (int)ctx->levels.size()) return STMG_EINVAL;
    const Level &L = *ctx->levels[level];
    if (k) *k = L.k;
    if (r) *r = L.r;
    if (n_cells)
        for (int a = 0; a < 3; ++a) n_cells[a] = L.n[a];
    if (n_total) *n_total = L.N;
    return STMG_OK;
}

static bool check_prec(stmg_ctx *ctx, int prec)
{
    return prec == ctx->mg->prec;
}

int stmg_set_state(stmg_ctx *ctx, const double *u_state)
{
    if (!ctx || !u_state) return fail(ctx, STMG_EINVAL, "NULL argument");
    return guarded(ctx, [&]() {
        mg_set_state(ctx, u_state);
        return STMG_OK;
    });
}

int stmg_level_state(stmg_ctx *ctx, int level, double *out)
{
    if (!ctx || !out || level < 0 || level >= (int)ctx->levels.size()) return fail(ctx, STMG_EINVAL, "invalid argument");
    return guarded(ctx, [&]() {
        if (!ctx->mg->state_set) return fail(ctx, STMG_ESTATE, "no state set");
        const Level &L = *ctx->levels[level];
        STMG_HIP(hipMemcpyAsync(out, ctx->mg->lv[level].st64.p, L.N * 8, hipMemcpyDeviceToDevice, ctx->stream));
        return STMG_OK;
    });
}

int stmg_smoother_rebuild(stmg_ctx *ctx, const double *u_state)
{
    if (!ctx || !u_state) return fail(ctx, STMG_EINVAL, "NULL argument");
    return guarded(ctx, [&]() {
        mg_set_state(ctx, u_state);
        mg_rebuild(ctx);
        return STMG_OK;
    });
}

int stmg_level_patch(stmg_ctx *ctx, int level, int cell, int prec, void *out)
{
    if (!ctx || !out || level < 0 || level + 1 >= (int)ctx->levels.size()) return fail(ctx, STMG_EINVAL, "invalid argument");
    return guarded(ctx, [&]() {
        MgLevel &M = ctx->mg->lv[level];
        Level &L = *M.L;
        if (cell < 0 || cell >= L.ncell) return fail(ctx, STMG_EINVAL, "cell out of range");
        if (!M.have_patches) return fail(ctx, STMG_ESTATE, "smoother not built (call stmg_smoother_rebuild)");
        if (prec != ctx->mg->prec) return fail(ctx, STMG_EINVAL, "prec must equal the multigrid precision");
        auto run = [&](auto tag) {
            using T = decltype(tag);
            PatchArgs<T, T> pa{};
            pa.n0 = L.n[0];
            pa.n1 = L.n[1];
            pa.n2 = L.n[2];
            pa.nt = L.nt;
            pa.elem = M.elem.as<T>();
            pa.rec_words = elem_record_words(L.dim, L.r);
            for (int i = 0; i < L.nt * L.nt; ++i) pa.K[i] = L.tc.K[i];
            for (int i = 0; i < L.nt; ++i) pa.w[i] = L.tc.w[i];
            pa.patches = (T *)out;
            pa.cell0 = cell;
            STMG_HIP((launch_patch<T, T>(L.dim, L.r, pa, 1, ctx->stream)));
            STMG_HIP(hipStreamSynchronize(ctx->stream));
        };
        if (prec == STMG_F64) run(double(0));
        else run(float(0));
        return STMG_OK;
    });
}

int stmg_batched_lu(int prec, void *A, const long long *a_off, const int *m_of, int batch, int *piv,
                    const long long *p_off, int *info, void *stream)
{
    return batched_lu_run(prec, A, a_off, m_of, batch, piv, p_off, info, nullptr, nullptr, stream, false,
                          MetaStaging::PerCall);
}

int stmg_batched_lu_config(int prec, void *A, const long long *a_off, const int *m_of, int batch, int *piv,
                           const long long *p_off, int *info, int wg_per_cu, int threads, const int *nb_by_class,
                           void *stream)
{
    if (wg_per_cu < 0 || wg_per_cu > 4 || (wg_per_cu > 0 && !nb_by_class)) return STMG_EINVAL;
    if (threads != 256 && threads != 512) return STMG_EINVAL;
    LuTune t{wg_per_cu, threads, {16, 16, 16, 16, 16}};
    if (wg_per_cu > 0)
        for (int c = 0; c < LU_TUNE_CLASSES; ++c) {
            const int nb = nb_by_class[c];
            if (nb != 4 && nb != 8 && nb != 16) return STMG_EINVAL;
            t.nb[c] = nb;
        }
    return batched_lu_run(prec, A, a_off, m_of, batch, piv, p_off, info, nullptr, nullptr, stream, false,
                          MetaStaging::PerCall, &t);
}

int stmg_batched_lu_noalloc(int prec, void *A, const long long *a_off, const int *m_of, int batch, int *piv,
                            const long long *p_off, int *info, void *stream)
{
    return batched_lu_run(prec, A, a_off, m_of, batch, piv, p_off, info, nullptr, nullptr, stream, false,
                          MetaStaging::Fixed);
}

int stmg_batched_lu_solve(int prec, const void *LU, const long long *a_off, const int *m_of, int batch,
                          const int *piv, const long long *p_off, void *b, const long long *b_off, void *stream)
{
    if (!b || !b_off) return STMG_EINVAL;
    return batched_lu_run(prec, const_cast<void *>(LU), a_off, m_of, batch, const_cast<int *>(piv), p_off, nullptr,
                          b, b_off, stream, true, MetaStaging::PerCall);
}

int stmg_level_jacobian_vmult(stmg_ctx *ctx, int level, int prec, const void *x, void *y)
{
    if (!ctx || !x || !y || level < 0 || level >= (int)ctx->levels.size()) return fail(ctx, STMG_EINVAL, "invalid argument");
    return guarded(ctx, [&]() {
        if (!ctx->mg->state_set) return fail(ctx, STMG_ESTATE, "no state set");
        Level &L = *ctx->levels[level];
        MgLevel &M = ctx->mg->lv[level];
        if (prec == STMG_F64)
            L.apply<double>(Mode::Jac, M.st64.as<double>(), (const double *)x, (double *)y, nullptr, nullptr, 1, ctx->stream);
        else if (prec == STMG_F32 && ctx->mg->prec == STMG_F32)
            L.apply<float>(Mode::Jac, M.st32.as<float>(), (const float *)x, (float *)y, nullptr, nullptr, 1, ctx->stream);
        else
            return fail(ctx, STMG_EINVAL, "precision not available on this context");
        return STMG_OK;
    });
}

int stmg_vanka_smooth(stmg_ctx *ctx, int level, int prec, const void *r, void *d, int sweeps)
{
    if (!ctx || !r || !d || level < 0 || level + 1 >= (int)ctx->levels.size() || sweeps < 0)
        return fail(ctx, STMG_EINVAL, "invalid argument (smoothing runs on every level but the coarsest)");
    return guarded(ctx, [&]() {
        if (!check_prec(ctx, prec)) return fail(ctx, STMG_EINVAL, "prec must equal the multigrid precision");
        if (!ctx->mg->lv[level].have_patches) return fail(ctx, STMG_ESTATE, "smoother not built (call stmg_smoother_rebuild)");
        for (int i = 0; i < sweeps; ++i) {
            if (prec == STMG_F64) mg_smooth<double>(ctx, level, (const double *)r, (double *)d);
            else mg_smooth<float>(ctx, level, (const float *)r, (float *)d);
        }
        return STMG_OK;
    });
}

int stmg_vcycle(stmg_ctx *ctx, int prec, const void *r, void *d)
{
    if (!ctx || !r || !d) return fail(ctx, STMG_EINVAL, "NULL argument");
    return guarded(ctx, [&]() {
        if (!check_prec(ctx, prec)) return fail(ctx, STMG_EINVAL, "prec must equal the multigrid precision");
        if (ctx->levels.size() > 1 && !ctx->mg->lv[0].have_patches)
            return fail(ctx, STMG_ESTATE, "smoother not built (call stmg_smoother_rebuild)");
        if (!ctx->mg->state_set) return fail(ctx, STMG_ESTATE, "no state set");
        if (prec == STMG_F64) mg_vcycle<double>(ctx, 0, (const double *)r, (double *)d);
        else mg_vcycle<float>(ctx, 0, (const float *)r, (float *)d);
        return STMG_OK;
    });
}

int stmg_prolongate(stmg_ctx *ctx, int level, int prec, const void *xc, void *yf)
{
    if (!ctx || !xc || !yf || level < 0 || level + 1 >= (int)ctx->levels.size()) return fail(ctx, STMG_EINVAL, "invalid argument");
    return guarded(ctx, [&]() {
        const Level &F = *ctx->levels[level], &C = *ctx->levels[level + 1];
        if (prec == STMG_F64) ctx->mg->tr[level]->prolongate<double>(F, C, (const double *)xc, (double *)yf, 0.0, ctx->stream);
        else ctx->mg->tr[level]->prolongate<float>(F, C, (const float *)xc, (float *)yf, 0.0f, ctx->stream);
        return STMG_OK;
    });
}

int stmg_restrict(stmg_ctx *ctx, int level, int prec, const void *xf, void *yc)
{
    if (!ctx || !xf || !yc || level < 0 || level + 1 >= (int)ctx->levels.size()) return fail(ctx, STMG_EINVAL, "invalid argument");
    return guarded(ctx, [&]() {
        const Level &F = *ctx->levels[level], &C = *ctx->levels[level + 1];
        if (prec == STMG_F64) ctx->mg->tr[level]->restrict_<double>(F, C, (const double *)xf, (double *)yc, ctx->stream);
        else ctx->mg->tr[level]->restrict_<float>(F, C, (const float *)xf, (float *)yc, ctx->stream);
        return STMG_OK;
    });
}

int stmg_fgmres(stmg_ctx *ctx, const double *u_state, const double *b, double *x, double rtol, int maxit, int *its,
                double *hist)
{
    if (!ctx || !u_state || !b || !x || maxit < 1) return fail(ctx, STMG_EINVAL, "invalid argument");
    return guarded(ctx, [&]() {
        if (ctx->levels.size() > 1 && !ctx->mg->lv[0].have_patches)
            return fail(ctx, STMG_ESTATE, "smoother not built (call stmg_smoother_rebuild)");
        FgmresOut o = fgmres(ctx, u_state, b, x, rtol, maxit);
        if (its) *its = o.its;
        if (hist)
            for (size_t i = 0; i < o.hist.size(); ++i) hist[i] = o.hist[i];
        return o.converged ? STMG_OK : STMG_NOT_CONVERGED;
    });
}

int stmg_newton_gmres_solve(stmg_ctx *ctx, double *u_inout, stmg_stats *stats)
{
    if (!ctx || !u_inout) return fail(ctx, STMG_EINVAL, "NULL argument");
    return guarded(ctx, [&]() { return newton_solve(ctx, u_inout, stats); });
}

int stmg_march(stmg_ctx *ctx, int nslabs, const double *rhs, long long rhs_stride, const double *v0, double *u,
               long long u_stride, stmg_stats *stats)
{
    if (!ctx || !u || nslabs < 0) return fail(ctx, STMG_EINVAL, "invalid argument");
    const Level &L = *ctx->levels[0];
    if (u_stride < L.N || (rhs && rhs_stride < L.N)) return fail(ctx, STMG_EINVAL, "stride below the slab size");
    int worst = STMG_OK;
    for (int n = 0; n < nslabs; ++n) {
        double *un = u + (long long)n * u_stride;
        // velocity at the end of the previous slab: its last time node
        const double *vp = n == 0 ? v0 : u + (long long)(n - 1) * u_stride + (long long)L.k * L.Nv1;
        int rc = stmg_set_slab_data(ctx, rhs ? rhs + (long long)n * rhs_stride : nullptr, vp);
        if (rc < 0) return rc;
        if (n > 0) {
            rc = guarded(ctx, [&]() {
                STMG_HIP(hipMemcpyAsync(un, un - u_stride, (size_t)L.N * 8, hipMemcpyDeviceToDevice, ctx->stream));
                return STMG_OK;
            });
            if (rc < 0) return rc;
        }
        rc = stmg_newton_gmres_solve(ctx, un, stats ? &stats[n] : nullptr);
        if (rc < 0) return rc;
        if (rc == STMG_NOT_CONVERGED) worst = rc;
    }
    return worst;
}

int stmg_timing_enable(stmg_ctx *ctx, int on)
{
    if (!ctx) return STMG_EINVAL;
    ctx->timers.on = on != 0;
    return STMG_OK;
}

int stmg_timing_reset(stmg_ctx *ctx)
{
    if (!ctx) return STMG_EINVAL;
    return guarded(ctx, [&]() {
        ctx->timers.flush();
        ctx->timers.acc.clear();
        return STMG_OK;
    });
}

int stmg_timing_get(stmg_ctx *ctx, const char *name, double *total_ms, long long *count)
{
    if (!ctx || !name) return STMG_EINVAL;
    return guarded(ctx, [&]() {
        ctx->timers.flush();
        double t = 0;
        long long c = 0;
        for (auto &kv : ctx->timers.acc)
            if (kv.first == name) {
                t = kv.second.first;
                c = kv.second.second;
            }
        if (total_ms) *total_ms = t;
        if (count) *count = c;
        return STMG_OK;
    });
}

} // extern "C"
