// Krylov and Newton drivers of the slab solve (Sec. "Inexact Newton-Krylov
// method"): right-preconditioned flexible GMRES in the M_n inner product
// (eq. lin-sys, eq. inexact) and the inexact Newton iteration with the
// Eisenstat-Walker forcing term (eq. ew), the nonmonotone Armijo line search
// (eq. armijo) and the smoother rebuild criteria (the remark after Lemma
// "patch perturbation").  All vector work and the Givens bookkeeping of
// FGMRES run on the device in FP64; the host reads back one residual estimate
// per Krylov iteration for the stopping test and a few scalars per Newton step.
#include "mg.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>

namespace stmg {

namespace {

bool verbose_newton()
{
    static int v = -1;
    if (v < 0) {
        const char *e = std::getenv("STMG_VERBOSE");
        v = (e && *e && *e != '0') ? 1 : 0;
    }
    return v == 1;
}

} // namespace

// ---------------------------------------------------------------------------
// FGMRES
// ---------------------------------------------------------------------------
FgmresOut fgmres(stmg_ctx *ctx, const double *state, const double *b, double *x, double rtol, int maxit)
{
    Level &L = *ctx->levels[0];
    const long long N = L.N;
    hipStream_t s = ctx->stream;
    Krylov &K = ctx->kry;
    K.ensure(N, maxit);
    double *V = K.V.as<double>(), *MV = K.MV.as<double>(), *Z = K.Z.as<double>();
    double *w = K.w.as<double>(), *u = K.u.as<double>(), *h = K.h.as<double>(), *part = K.partial.as<double>();
    double *H = K.H.as<double>(), *cs = K.cs.as<double>(), *sn = K.sn.as<double>(), *g = K.g.as<double>();
    double *report = K.report.as<double>();
    const int ldh = K.maxit;   // column stride of H is ldh + 1
    FgmresOut out;
    STMG_HIP(hipMemcpyAsync(V, b, N * 8, hipMemcpyDeviceToDevice, s));
    L.apply<double>(Mode::Mass, nullptr, V, MV, nullptr, nullptr, 1, s);
    STMG_HIP(vec_multidot(N, 1, MV, V, N, h, part, 0, s));
    double beta2 = 0;
    STMG_HIP(hipMemcpyAsync(&beta2, h, 8, hipMemcpyDeviceToHost, s));
    STMG_HIP(hipStreamSynchronize(s));
    const double beta = std::sqrt(std::max(beta2, 0.0));
    out.hist.push_back(beta);
    if (beta == 0.0) {
        STMG_HIP(vec_fill<double>(N, 0.0, x, s));
        out.converged = true;
        return out;
    }
    STMG_HIP(vec_axpby<double>(N, 1.0 / beta, V, 0.0, V, s));
    STMG_HIP(vec_axpby<double>(N, 1.0 / beta, MV, 0.0, MV, s));
    STMG_HIP(vec_fill<double>(ldh + 1, 0.0, g, s));
    STMG_HIP(hipMemcpyAsync(g, &beta, 8, hipMemcpyHostToDevice, s));
    int its = 0;
    double rep[2] = {0, 0};
    for (int j = 0; j < maxit; ++j) {
        double *vj = V + (long long)j * N, *zj = Z + (long long)j * N;
        mg_precondition(ctx, vj, zj);
        L.apply<double>(Mode::Jac, state, zj, w, nullptr, nullptr, 1, s);
        L.apply<double>(Mode::Mass, nullptr, w, u, nullptr, nullptr, 1, s);
        // classical Gram-Schmidt in the M inner product, twice
        double *h1 = h, *h2 = h + (ldh + 1), *hn = h + 2 * (ldh + 1);
        STMG_HIP(vec_multidot(N, j + 1, u, V, N, h1, part, 0, s));
        STMG_HIP(vec_subtract_combination(N, j + 1, h1, V, N, w, s));
        STMG_HIP(vec_subtract_combination(N, j + 1, h1, MV, N, u, s));
        STMG_HIP(vec_multidot(N, j + 1, u, V, N, h2, part, 0, s));
        STMG_HIP(vec_subtract_combination(N, j + 1, h2, V, N, w, s));
        STMG_HIP(vec_subtract_combination(N, j + 1, h2, MV, N, u, s));
        STMG_HIP(vec_multidot(N, 1, u, w, N, hn, part, 0, s));
        STMG_HIP(krylov_givens_column(j, ldh, h1, h2, hn, H, cs, sn, g, report, s));
        STMG_HIP(hipMemcpyAsync(rep, report, sizeof(rep), hipMemcpyDeviceToHost, s));
        STMG_HIP(hipStreamSynchronize(s));
        its = j + 1;
        const double res = rep[0], sub = rep[1];
        out.hist.push_back(res);
        if (res <= rtol * beta || sub == 0.0) {
            out.converged = res <= rtol * beta;
            break;
        }
        STMG_HIP(vec_axpby<double>(N, 1.0 / sub, w, 0.0, V + (long long)(j + 1) * N, s));
        STMG_HIP(vec_axpby<double>(N, 1.0 / sub, u, 0.0, MV + (long long)(j + 1) * N, s));
    }
    STMG_HIP(krylov_upper_solve(its, ldh, H, g, K.y.as<double>(), s));
    STMG_HIP(vec_combination(N, its, K.y.as<double>(), Z, N, x, s));
    STMG_HIP(hipStreamSynchronize(s));
    out.its = its;
    return out;
}

// ---------------------------------------------------------------------------
// Newton control
// ---------------------------------------------------------------------------
namespace {

constexpr double NORM_FLOOR = 1e-30;   // the eps of eq. ew

// Eisenstat-Walker forcing term of the next linear solve (eq. ew): the ratio
// of the current to the previous residual M-norm raised to theta; the factor
// c_eta multiplies the previous forcing term and the result is held in
// [eta_min, eta_max] (the form of the appendix's Newton algorithm, whose
// parameter names Sec. "Numerical experiments" uses).
double forcing_term(double eta_prev, double res, double res_prev, const stmg_options &o)
{
    const double ratio = res / std::max(res_prev, NORM_FLOOR);
    return std::min(std::max(o.ew_c * eta_prev * std::pow(ratio, o.ew_theta), o.ew_eta_min), o.ew_eta_max);
}

// Nonmonotone reference of the line search (Grippo-Lampariello-Lucidi): the
// largest of the last `size` accepted merit values of the slab's Newton
// iteration, seeded with the initial one; size 0 = the monotone rule.
struct MeritMemory {
    int size;
    std::vector<double> values;
    MeritMemory(double phi_initial, int size_) : size(size_), values{phi_initial} {}
    double reference(double phi0) const
    {
        return size > 0 ? *std::max_element(values.begin(), values.end()) : phi0;
    }
    void remember(double phi)
    {
        if (size <= 0) return;
        values.push_back(phi);
        if ((int)values.size() > size) values.erase(values.begin(), values.end() - size);
    }
};

// Local minimizer of the polynomial model of the merit function along the
// Newton direction: the quadratic phi0 + g0 a + b a^2 through the last
// rejected step, after later rejections the cubic phi0 + g0 a + b a^2 + c a^3
// through the last two.  false when the model has none.
bool model_minimizer(double phi0, double g0, const std::vector<std::pair<double, double>> &failures, double &out)
{
    const double a1 = failures.back().first, p1 = failures.back().second;
    if (failures.size() == 1) {
        const double curv = p1 - phi0 - g0 * a1;
        if (curv <= 0.0) return false;
        out = -g0 * a1 * a1 / (2.0 * curv);
        return true;
    }
    const double a2 = failures[failures.size() - 2].first, p2 = failures[failures.size() - 2].second;
    const double e1 = p1 - phi0 - g0 * a1, e2 = p2 - phi0 - g0 * a2;
    const double det = a1 * a1 * a2 * a2 * (a1 - a2);
    if (det == 0.0) return false;
    const double c3 = (a2 * a2 * e1 - a1 * a1 * e2) / det;
    const double b2 = (a1 * a1 * a1 * e2 - a2 * a2 * a2 * e1) / det;
    if (c3 == 0.0) {
        if (b2 <= 0.0) return false;
        out = -g0 / (2.0 * b2);
        return true;
    }
    const double disc = b2 * b2 - 3.0 * c3 * g0;   // critical points of the cubic
    if (disc < 0.0) return false;
    out = (-b2 + std::sqrt(disc)) / (3.0 * c3);
    return true;
}

// Step length by the nonmonotone Armijo condition (eq. armijo against the
// remembered reference).  merit(a) evaluates phi(a) = 1/2 ||R(U + a dU)||_M^2.
// A rejected step is replaced by the model minimizer held in [0.1 a, 0.5 a]
// (ls_tau a when there is none); after ls_max_backtracks rejections, or once
// the step would reach ls_alpha_min, the step is ls_alpha_min.
template <typename Merit>
double line_search(Merit &&merit, double phi0, double g0, MeritMemory &memory, const stmg_options &o, int &rejected)
{
    double alpha = o.ls_lambda0;
    std::vector<std::pair<double, double>> failures;
    while (alpha > o.ls_alpha_min) {
        const double phit = merit(alpha);
        if (std::isfinite(phit) && phit <= memory.reference(phi0) + o.ls_c * alpha * g0) {
            memory.remember(phit);
            rejected = (int)failures.size();
            return alpha;
        }
        failures.push_back({alpha, phit});
        if ((int)failures.size() > o.ls_max_backtracks) break;
        double trial = 0;
        if (!model_minimizer(phi0, g0, failures, trial) || !std::isfinite(trial)) alpha = o.ls_tau * alpha;
        else alpha = std::min(std::max(trial, 0.1 * alpha), 0.5 * alpha);
    }
    rejected = (int)failures.size();
    return o.ls_alpha_min;
}

// s consecutive FGMRES residual ratios r_{j+1} / r_j of at least theta
bool fgmres_stagnated(const std::vector<double> &hist, int s, double theta)
{
    int run = 0;
    for (size_t i = 0; i + 1 < hist.size(); ++i) {
        if (hist[i] <= 0) continue;
        run = hist[i + 1] / hist[i] >= theta ? run + 1 : 0;
        if (run >= s) return true;
    }
    return false;
}

// When the midpoint-frozen smoother is rebuilt (the criteria of the remark
// after Lemma "patch perturbation", thresholds from the options).  Before a
// Newton step: when none is built yet, on Newton deterioration (last residual
// contraction rho >= theta_N) or on linear deterioration (last FGMRES count
// kappa >= max(theta_L kappa_ref, kappa_abs), kappa_ref = the count at the
// last such rebuild).  After a step: when its FGMRES residuals stagnated.
struct RebuildPolicy {
    const stmg_options &o;
    double rho = 1.0;
    int kappa = 1, kappa_ref = 1;
    bool built = false;
    explicit RebuildPolicy(const stmg_options &o_) : o(o_) {}
    bool due_before_step() const
    {
        return !built || rho >= o.rb_theta_N || kappa >= std::max(o.rb_theta_L * kappa_ref, o.rb_kappa_abs);
    }
    void rebuilt_before_step()
    {
        built = true;
        kappa_ref = std::max(1, kappa);
    }
    void record_step(double res, double res_prev, int fgmres_its)
    {
        rho = res / std::max(res_prev, NORM_FLOOR);
        kappa = std::max(1, fgmres_its);
    }
    bool due_after_step(const std::vector<double> &hist) const
    {
        return fgmres_stagnated(hist, o.rb_stag_s, o.rb_stag_theta);
    }
};

} // namespace

// ---------------------------------------------------------------------------
// Newton
// ---------------------------------------------------------------------------
int newton_solve(stmg_ctx *ctx, double *U, stmg_stats *stats)
{
    const auto t0 = std::chrono::steady_clock::now();
    Level &L = *ctx->levels[0];
    Mg &mg = *ctx->mg;
    const stmg_options &o = ctx->opt;
    const long long N = L.N;
    hipStream_t s = ctx->stream;
    Krylov &W = ctx->kry;
    const double *rhs = ctx->has_rhs ? ctx->rhs.as<double>() : nullptr;
    const double *vprev = ctx->has_vprev ? ctx->vprev.as<double>() : nullptr;
    W.ensure(N, std::max(1, o.fgmres_maxit));
    double *part = W.partial.as<double>();
    double *r = W.r.as<double>(), *dU = W.dU.as<double>(), *tmp = W.tmp.as<double>();
    auto dot = [&](const double *a, const double *b) {
        STMG_HIP(vec_multidot(N, 1, a, b, N, W.dot.as<double>(), part, 0, s));
        double v = 0;
        STMG_HIP(hipMemcpyAsync(&v, W.dot.p, 8, hipMemcpyDeviceToHost, s));
        STMG_HIP(hipStreamSynchronize(s));
        return v;
    };
    auto residual = [&](const double *X, double *R) { L.apply<double>(Mode::Res, nullptr, X, R, rhs, vprev, 1, s); };
    auto mnorm = [&](const double *v) {
        L.apply<double>(Mode::Mass, nullptr, v, tmp, nullptr, nullptr, 1, s);
        return std::sqrt(std::max(dot(v, tmp), 0.0));
    };
    stmg_stats st{};
    residual(U, r);
    double res = mnorm(r);
    if (!std::isfinite(res)) {
        ctx->err = "non-finite initial residual";
        return STMG_ENONFINITE;
    }
    st.res0_M = res;
    const double target = std::max(o.newton_atol, o.newton_rtol * res);
    MeritMemory memory(0.5 * res * res, o.ls_window);
    RebuildPolicy policy(o);
    double eta = o.ew_eta0, res_before = res;
    for (size_t l = 0; l < mg.lv.size(); ++l) mg.lv[l].have_patches = false;
    int k = 0;
    while (res > target && k < o.newton_maxit) {
        mg_set_state(ctx, U);
        if (policy.due_before_step()) {
            mg_rebuild(ctx);
            st.rebuilds++;
            policy.rebuilt_before_step();
        }
        if (k > 0) eta = forcing_term(eta, res, res_before, o);
        // the correction: J dU = -R to the relative accuracy eta (eq. inexact)
        STMG_HIP(vec_axpby<double>(N, -1.0, r, 0.0, W.rt.as<double>(), s));
        const FgmresOut lin = fgmres(ctx, U, W.rt.as<double>(), dU, eta, o.fgmres_maxit);
        if (k < 64) st.fgmres_its[k] = lin.its;
        st.fgmres_its_total += lin.its;
        // phi'(0) = (M R)^T (J dU)
        L.apply<double>(Mode::Mass, nullptr, r, W.Mr.as<double>(), nullptr, nullptr, 1, s);
        L.apply<double>(Mode::Jac, U, dU, tmp, nullptr, nullptr, 1, s);
        const double g0 = dot(tmp, W.Mr.as<double>());
        auto merit = [&](double a) {
            double *Ut = W.Ut.as<double>(), *rt = W.rt.as<double>();
            STMG_HIP(hipMemcpyAsync(Ut, U, N * 8, hipMemcpyDeviceToDevice, s));
            STMG_HIP(vec_axpby<double>(N, a, dU, 1.0, Ut, s));
            residual(Ut, rt);
            const double m = mnorm(rt);
            return 0.5 * m * m;
        };
        int rejected = 0;
        const double alpha = line_search(merit, 0.5 * res * res, g0, memory, o, rejected);
        st.backtracks += rejected;
        STMG_HIP(vec_axpby<double>(N, alpha, dU, 1.0, U, s));
        res_before = res;
        residual(U, r);
        res = mnorm(r);
        if (!std::isfinite(res)) {
            ctx->err = "non-finite residual";
            return STMG_ENONFINITE;
        }
        policy.record_step(res, res_before, lin.its);
        if (policy.due_after_step(lin.hist)) {
            mg_set_state(ctx, U);
            mg_rebuild(ctx);
            st.rebuilds++;
        }
        ++k;
        if (verbose_newton()) {
            std::fprintf(stderr,
                         "[stmg] newton %d: |R|_M %.3e (rho %.3f) fgmres %d (eta %.2e reached %.2e) alpha %.3g "
                         "rebuilds %d  %.2f s\n",
                         k, res, policy.rho, lin.its, eta, lin.hist.back() / lin.hist.front(), alpha, st.rebuilds,
                         std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
            std::fflush(stderr);
        }
    }
    STMG_HIP(hipStreamSynchronize(s));
    st.newton_its = k;
    st.res_M = res;
    st.wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    return res <= target ? STMG_OK : STMG_NOT_CONVERGED;
}

} // namespace stmg
