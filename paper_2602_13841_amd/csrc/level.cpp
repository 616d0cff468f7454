// Level set-up and dispatch of the cell operators.
#include "context.h"

#include <cmath>
#include <algorithm>
#include <cstring>

namespace stmg {

static long long binom(int n, int k)
{
    long long r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

void Level::init(const stmg_problem &p, int k_, int r_, int nx, int ny, int nz, int nq_,
                 const std::vector<double> &verts)
{
    dim = p.dim;
    n[0] = nx;
    n[1] = ny;
    n[2] = dim == 3 ? nz : 1;
    r = r_;
    k = k_;
    nq = nq_ > 0 ? nq_ : default_nq(r);
    nt = k + 1;
    npm = (int)binom(r + dim, dim);
    dmask = p.dirichlet_faces;
    nu = p.nu;
    tau = p.tau;
    g1 = p.gamma1;
    g2 = p.gamma2;
    ncell = (long long)n[0] * n[1] * n[2];
    Nn = 1;
    for (int a = 0; a < dim; ++a) Nn *= (long long)(r + 1) * n[a] + 1;
    Nv1 = dim * Nn;
    Np1 = ncell * npm;
    N = nt * (Nv1 + Np1);
    nl = 1;
    for (int a = 0; a < dim; ++a) nl *= r + 2;
    tc = time_coefficients(k, tau);
    lay.init(r, nq);
    std::vector<double> tb = build_table_block(r, nq, lay);
    std::vector<float> tbf(tb.begin(), tb.end());
    const bool dry = arena_counting();   // measuring only: no device work
    tab64.alloc(tb.size() * sizeof(double));
    tab32.alloc(tbf.size() * sizeof(float));
    if (!dry) {
        STMG_HIP(hipMemcpy(tab64.p, tb.data(), tb.size() * sizeof(double), hipMemcpyHostToDevice));
        STMG_HIP(hipMemcpy(tab32.p, tbf.data(), tbf.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    {
        std::vector<int> bc;
        for (long long c = 0; c < ncell; ++c) {
            const int cc[3] = {(int)(c % n[0]), (int)((c / n[0]) % n[1]), (int)(c / ((long long)n[0] * n[1]))};
            bool b = false;
            for (int a = 0; a < dim; ++a) b = b || cc[a] == 0 || cc[a] == n[a] - 1;
            if (b) bc.push_back((int)c);
        }
        nbcell = (int)bc.size();
        bcells.alloc(std::max<size_t>(bc.size(), 1) * sizeof(int));
        if (!bc.empty() && !dry)
            STMG_HIP(hipMemcpy(bcells.p, bc.data(), bc.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    mapped = !verts.empty();
    vert_host = verts;
    if (mapped) {
        vert.alloc(verts.size() * sizeof(double));
        if (!dry) STMG_HIP(hipMemcpy(vert.p, verts.data(), verts.size() * sizeof(double), hipMemcpyHostToDevice));
    }
}

void Level::alloc_work(int nvec64, int nvec32)
{
    const size_t cellw = (size_t)ncell * nt * dim * nl;
    nvec_cap64 = nvec64;
    nvec_cap32 = nvec32;
    if (nvec64 > 0) E64.alloc(nvec64 * cellw * 8);
    if (nvec32 > 0) E32.alloc(nvec32 * cellw * 4);
}

template <typename T> CellArgs<T> Level::cell_args() const
{
    CellArgs<T> a{};
    a.n0 = n[0];
    a.n1 = n[1];
    a.n2 = n[2];
    a.nt = nt;
    a.ncell = (int)ncell;
    a.Nn = Nn;
    a.Nv1 = Nv1;
    a.Np1 = Np1;
    a.Nslab = N;
    a.tab = std::is_same<T, double>::value ? (const T *)tab64.p : (const T *)tab32.p;
    a.vert = mapped ? vert.as<double>() : nullptr;
    a.mapped = mapped ? 1 : 0;
    a.dmask = dmask;
    a.bcells = bcells.as<int>();
    a.nbcell = nbcell;
    a.nu = (T)nu;
    a.g1 = (T)g1;
    a.g2 = (T)g2;
    for (int i = 0; i < nt * nt; ++i) a.K[i] = (T)tc.K[i];
    for (int i = 0; i < nt; ++i) {
        a.w[i] = (T)tc.w[i];
        a.phi0[i] = (T)tc.phi0[i];
    }
    return a;
}

template <typename T> GatherArgs<T> Level::gather_args() const
{
    GatherArgs<T> g{};
    g.n0 = n[0];
    g.n1 = n[1];
    g.n2 = n[2];
    g.r = r;
    g.nt = nt;
    g.dim = dim;
    g.Nn = Nn;
    g.Nv1 = Nv1;
    g.Nslab = N;
    g.nl = nl;
    g.alpha = T(1);
    g.accumulate = 0;
    g.inv_mult = 0;
    return g;
}

template <typename T>
void Level::apply(Mode mode, const T *state, const T *x, T *y, const T *rhs, const T *vprev, int nvec,
                  hipStream_t s)
{
    const bool f64 = std::is_same<T, double>::value;
    // the work buffers were sized at creation for cap vectors per launch:
    // larger batches run in chunks of cap vectors
    const int cap = f64 ? nvec_cap64 : nvec_cap32;
    if (cap < 1) throw HipError("operator precision not prepared on this level", STMG_EINVAL);
    if (nvec > cap) {
        for (int v0 = 0; v0 < nvec; v0 += cap) {
            const int nv = std::min(cap, nvec - v0);
            apply<T>(mode, state, x + (long long)v0 * N, y + (long long)v0 * N, rhs, vprev, nv, s);
        }
        return;
    }
    DevBuf &Eb = f64 ? E64 : E32;
    Eb.require((size_t)nvec * ncell * nt * dim * nl * sizeof(T), "E");
    const bool faces = mode != Mode::Mass && nbcell > 0;
    CellArgs<T> a = cell_args<T>();
    a.x = x;
    a.state = state;
    a.vprev = vprev;
    a.rhs = rhs;
    a.E = Eb.as<T>();
    a.y = y;
    a.xstride = N;
    a.ystride = N;
    a.sstride = 0;
    static const char *names64[3] = {"cell_jac_f64", "cell_res_f64", "cell_mass_f64"};
    static const char *names32[3] = {"cell_jac_f32", "cell_res_f32", "cell_mass_f32"};
    const char *nm = f64 ? names64[(int)mode] : names32[(int)mode];
    // 3D Jacobian: the boundary faces run in the same launch as the volume
    const bool fused = mode == Mode::Jac && dim == 3 && jac_fuse_faces(r, nq, f64);
    {
        TimerScope ts(timers, nm, s);
        if (fused) STMG_HIP(launch_jac_fused_op<T>(r, nq, a, nvec, s));
        else STMG_HIP(launch_cell_op<T>(mode, dim, r, nq, a, nvec, s));
    }
    if (faces && !fused) {
        static const char *fn64[2] = {"face_jac_f64", "face_res_f64"};
        static const char *fn32[2] = {"face_jac_f32", "face_res_f32"};
        TimerScope ts(timers, f64 ? fn64[(int)mode] : fn32[(int)mode], s);
        STMG_HIP(launch_face_op<T>(mode, dim, r, nq, a, nvec, s));
    }
    GatherArgs<T> g = gather_args<T>();
    g.E = Eb.as<T>();
    g.rhs = rhs;
    g.y = y;
    g.ystride = N;
    {
        TimerScope ts(timers, f64 ? "gather_f64" : "gather_f32", s);
        STMG_HIP(launch_gather<T>(g, nvec, s));
    }
}

template CellArgs<double> Level::cell_args<double>() const;
template GatherArgs<double> Level::gather_args<double>() const;
template GatherArgs<float> Level::gather_args<float>() const;
template CellArgs<float> Level::cell_args<float>() const;
template void Level::apply<double>(Mode, const double *, const double *, double *, const double *, const double *,
                                   int, hipStream_t);
template void Level::apply<float>(Mode, const float *, const float *, float *, const float *, const float *, int,
                                  hipStream_t);

} // namespace stmg
