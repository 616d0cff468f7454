// Grid transfers of the hp space-time hierarchy (Sec. "Grid transfer
// operators", eq. MatGeomProl).
//
// Prolongation = canonical embedding of the coarse space into the fine one,
// evaluated cell by cell in reference coordinates:
//   h-step (n -> 2n cells, same (k, r)): a fine cell is the child o of its
//          coarse parent, xi_coarse = (o + xi_fine)/2 per axis;
//   p-step (same mesh, (kc, rc) -> (k, r)): the coarse Q_{rc+1} field at the
//          fine Gauss-Lobatto nodes, the coarse modes embedded in the fine
//          modal basis (same orthonormal functions), the coarse DG(kc) time
//          polynomial at the fine Radau nodes.
// Pressure of an h-step: the coarse polynomial restricted to a child is
// expanded in the fine orthonormal basis (exact L2 projection, tensor
// product of 1D Gauss integrals).  Restriction = transpose.  Level states are
// transferred by evaluating the finer field at the coarser nodes.
//
// The spatial maps are built on the host as CSR matrices over scalar nodes
// (one matrix serves all components and time nodes) and applied on the
// device by kron_csr_apply.
#include "transfers.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <stdexcept>

namespace stmg {

namespace {

struct Entry {
    long long col;
    double val;
};

// lattice coordinate g along an axis -> (cell, local Gauss-Lobatto index);
// interface nodes go to the cell above them, the last node to the last cell
void locate(long long g, int r, int ncell, int &cell, int &loc)
{
    cell = (int)(g / (r + 1));
    loc = (int)(g - (long long)(r + 1) * cell);
    if (cell >= ncell) {
        cell = ncell - 1;
        loc = r + 1;
    }
}

HostCsr tensor_csr(int dim, const std::vector<std::vector<std::vector<Entry>>> &axes, const long long Nrow[3],
                   const long long Ncol[3], bool count_only)
{
    HostCsr A;
    long long nrows = 1, ncols = 1;
    for (int a = 0; a < dim; ++a) {
        nrows *= Nrow[a];
        ncols *= Ncol[a];
    }
    // the device CSR kernels index rows, columns and entries with 32 bits
    if (nrows > INT_MAX || ncols > INT_MAX) throw std::invalid_argument("transfer matrix too large for 32-bit indices");
    A.nrows = (int)nrows;
    A.ncols = (int)ncols;
    if (count_only) {
        // a row's entries are the nonzero products of one nonzero 1D entry per
        // axis, so the total factorizes over the axes
        long long nnz = 1;
        for (int a = 0; a < dim; ++a) {
            long long s = 0;
            for (const auto &lst : axes[a])
                for (const Entry &e : lst) s += e.val != 0.0;
            nnz *= s;
        }
        if (nnz > INT_MAX) throw std::invalid_argument("transfer matrix has more than 2^31 - 1 entries");
        A.counted_nnz = nnz;
        return A;
    }
    A.rowptr.assign(nrows + 1, 0);
    std::vector<Entry> cur, nxt;
    for (long long row = 0; row < nrows; ++row) {
        long long gi[3] = {0, 0, 0}, rest = row;
        for (int a = 0; a < dim; ++a) {
            gi[a] = rest % Nrow[a];
            rest /= Nrow[a];
        }
        cur.assign(1, Entry{0, 1.0});
        long long stride = 1;
        for (int a = 0; a < dim; ++a) {
            nxt.clear();
            for (const Entry &e : cur)
                for (const Entry &f : axes[a][gi[a]]) nxt.push_back(Entry{e.col + stride * f.col, e.val * f.val});
            cur.swap(nxt);
            stride *= Ncol[a];
        }
        std::sort(cur.begin(), cur.end(), [](const Entry &x, const Entry &y) { return x.col < y.col; });
        if ((long long)A.col.size() + (long long)cur.size() > INT_MAX)
            throw std::invalid_argument("transfer matrix has more than 2^31 - 1 entries");
        for (const Entry &e : cur) {
            if (e.val == 0.0) continue;
            A.col.push_back((int)e.col);
            A.val.push_back(e.val);
        }
        A.rowptr[row + 1] = (int)A.col.size();
    }
    return A;
}

} // namespace

HostCsr transpose(const HostCsr &A)
{
    HostCsr B;
    B.nrows = A.ncols;
    B.ncols = A.nrows;
    if (A.counted_nnz >= 0) {
        B.counted_nnz = A.counted_nnz;
        return B;
    }
    B.rowptr.assign(B.nrows + 1, 0);
    for (int c : A.col) B.rowptr[c + 1]++;
    for (int i = 0; i < B.nrows; ++i) B.rowptr[i + 1] += B.rowptr[i];
    B.col.resize(A.col.size());
    B.val.resize(A.val.size());
    std::vector<int> pos(B.rowptr.begin(), B.rowptr.end() - 1);
    for (int r = 0; r < A.nrows; ++r)
        for (int k = A.rowptr[r]; k < A.rowptr[r + 1]; ++k) {
            int p = pos[A.col[k]]++;
            B.col[p] = r;
            B.val[p] = A.val[k];
        }
    return B;
}

HostCsr velocity_prolongation(const Level &f, const Level &c, char kind, bool count_only)
{
    std::vector<double> glf, glc;
    lobatto_points(f.r + 2, glf);
    lobatto_points(c.r + 2, glc);
    std::vector<std::vector<std::vector<Entry>>> axes(f.dim);
    long long Nf[3] = {1, 1, 1}, Nc[3] = {1, 1, 1};
    for (int a = 0; a < f.dim; ++a) {
        Nf[a] = (long long)(f.r + 1) * f.n[a] + 1;
        Nc[a] = (long long)(c.r + 1) * c.n[a] + 1;
        axes[a].resize(Nf[a]);
        for (long long g = 0; g < Nf[a]; ++g) {
            int cf, lf;
            locate(g, f.r, f.n[a], cf, lf);
            double xf = glf[lf], xc;
            int cc;
            if (kind == 'p') {
                cc = cf;
                xc = xf;
            } else {
                cc = cf / 2;
                xc = 0.5 * ((cf % 2) + xf);
            }
            std::vector<double> L, dL;
            lagrange_tables(glc, std::vector<double>{xc}, L, dL);
            for (int j = 0; j < c.r + 2; ++j) axes[a][g].push_back(Entry{(long long)(c.r + 1) * cc + j, L[j]});
        }
    }
    return tensor_csr(f.dim, axes, Nf, Nc, count_only);
}

HostCsr state_interpolation(const Level &f, const Level &c, char kind, bool count_only)
{
    std::vector<double> glf, glc;
    lobatto_points(f.r + 2, glf);
    lobatto_points(c.r + 2, glc);
    std::vector<std::vector<std::vector<Entry>>> axes(f.dim);
    long long Nf[3] = {1, 1, 1}, Nc[3] = {1, 1, 1};
    for (int a = 0; a < f.dim; ++a) {
        Nf[a] = (long long)(f.r + 1) * f.n[a] + 1;
        Nc[a] = (long long)(c.r + 1) * c.n[a] + 1;
        axes[a].resize(Nc[a]);
        for (long long g = 0; g < Nc[a]; ++g) {
            int cc, lc;
            locate(g, c.r, c.n[a], cc, lc);
            double xc = glc[lc], xf;
            int cf;
            if (kind == 'p') {
                cf = cc;
                xf = xc;
            } else {
                int o = std::min((int)std::floor(2.0 * xc), 1);
                cf = 2 * cc + o;
                xf = 2.0 * xc - o;
            }
            std::vector<double> L, dL;
            lagrange_tables(glf, std::vector<double>{xf}, L, dL);
            for (int j = 0; j < f.r + 2; ++j) axes[a][g].push_back(Entry{(long long)(f.r + 1) * cf + j, L[j]});
        }
    }
    return tensor_csr(f.dim, axes, Nc, Nf, count_only);
}

HostCsr pressure_prolongation(const Level &f, const Level &c, char kind, bool count_only)
{
    std::vector<int> mf = pressure_multi_indices(f.r, f.dim), mc = pressure_multi_indices(c.r, c.dim);
    int nf = (int)mf.size() / 3, nc = (int)mc.size() / 3;
    HostCsr A;
    A.nrows = (int)(f.ncell * nf);
    A.ncols = (int)(c.ncell * nc);
    if (count_only) A.counted_nnz = 0;
    else A.rowptr.assign(A.nrows + 1, 0);
    // 1D child integrals m1[o][alpha][beta] = int_0^1 L_alpha(s) L_beta((o+s)/2) ds
    int rmax = std::max(f.r, c.r);
    std::vector<double> gx, gw;
    gauss_rule(rmax + 2, gx, gw);
    std::vector<double> Lf, Lc[2];
    legendre01_table(f.r, gx, Lf);
    for (int o = 0; o < 2; ++o) {
        std::vector<double> xs(gx.size());
        for (size_t q = 0; q < gx.size(); ++q) xs[q] = 0.5 * (o + gx[q]);
        legendre01_table(c.r, xs, Lc[o]);
    }
    auto m1 = [&](int o, int al, int be) {
        double s = 0;
        for (size_t q = 0; q < gx.size(); ++q) s += gw[q] * Lf[q * (f.r + 1) + al] * Lc[o][q * (c.r + 1) + be];
        return s;
    };
    for (long long cell = 0; cell < f.ncell; ++cell) {
        int cf[3] = {(int)(cell % f.n[0]), (int)((cell / f.n[0]) % f.n[1]), f.dim == 3 ? (int)(cell / (f.n[0] * f.n[1])) : 0};
        long long ccell;
        if (kind == 'p') ccell = cell;
        else ccell = cf[0] / 2 + (long long)c.n[0] * (cf[1] / 2 + (long long)c.n[1] * (cf[2] / 2));
        for (int i = 0; i < nf; ++i) {
            long long row = cell * nf + i;
            for (int j = 0; j < nc; ++j) {
                double v;
                if (kind == 'p') {
                    v = (mf[3 * i] == mc[3 * j] && mf[3 * i + 1] == mc[3 * j + 1] && mf[3 * i + 2] == mc[3 * j + 2]) ? 1.0
                                                                                                                : 0.0;
                } else {
                    v = 1.0;
                    for (int a = 0; a < f.dim; ++a) v *= m1(cf[a] % 2, mf[3 * i + a], mc[3 * j + a]);
                }
                if (v != 0.0) {
                    if (count_only) {
                        ++A.counted_nnz;
                        continue;
                    }
                    A.col.push_back((int)(ccell * nc + j));
                    A.val.push_back(v);
                }
            }
            if (!count_only) A.rowptr[row + 1] = (int)A.col.size();
        }
    }
    return A;
}

void DevCsr::upload(const HostCsr &A)
{
    nrows = A.nrows;
    ncols = A.ncols;
    nnz = A.nnz();
    rowptr.alloc(sizeof(int) * (nrows + 1));
    col.alloc(sizeof(int) * std::max<long long>(nnz, 1));
    val64.alloc(sizeof(double) * std::max<long long>(nnz, 1));
    val32.alloc(sizeof(float) * std::max<long long>(nnz, 1));
    if (arena_counting()) return;
    std::vector<float> vf(A.val.begin(), A.val.end());
    STMG_HIP(hipMemcpy(rowptr.p, A.rowptr.data(), sizeof(int) * (nrows + 1), hipMemcpyHostToDevice));
    if (nnz) {
        STMG_HIP(hipMemcpy(col.p, A.col.data(), sizeof(int) * nnz, hipMemcpyHostToDevice));
        STMG_HIP(hipMemcpy(val64.p, A.val.data(), sizeof(double) * nnz, hipMemcpyHostToDevice));
        STMG_HIP(hipMemcpy(val32.p, vf.data(), sizeof(float) * nnz, hipMemcpyHostToDevice));
    }
}

static void upload_dense(DevBuf &b64, DevBuf &b32, const std::vector<double> &v)
{
    std::vector<float> f(v.begin(), v.end());
    b64.alloc(v.size() * sizeof(double));
    b32.alloc(v.size() * sizeof(float));
    if (arena_counting()) return;
    STMG_HIP(hipMemcpy(b64.p, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
    STMG_HIP(hipMemcpy(b32.p, f.data(), v.size() * sizeof(float), hipMemcpyHostToDevice));
}

void Transfer::build(const Level &f, const Level &c, char kind_)
{
    kind = kind_;
    const bool dry = arena_counting();
    HostCsr Pv = velocity_prolongation(f, c, kind, dry);
    HostCsr Pp = pressure_prolongation(f, c, kind, dry);
    vel.upload(Pv);
    velT.upload(transpose(Pv));
    pres.upload(Pp);
    presT.upload(transpose(Pp));
    state.upload(state_interpolation(f, c, kind, dry));
    std::vector<double> Pt = time_embedding(f.k, c.k);           // [a_f][b_c]
    std::vector<double> PtT(Pt.size());
    for (int a = 0; a < f.nt; ++a)
        for (int b = 0; b < c.nt; ++b) PtT[b * f.nt + a] = Pt[a * c.nt + b];
    upload_dense(Pt64, Pt32, Pt);
    upload_dense(PtT64, PtT32, PtT);
    // time interpolation of states: It[b_c][a_f] = phi^f_a(t^c_b)
    TimeCoefs tf = time_coefficients(f.k, 1.0), tc = time_coefficients(c.k, 1.0);
    std::vector<double> fs(tf.s, tf.s + tf.nt), cs(tc.s, tc.s + tc.nt), L, dL;
    lagrange_tables(fs, cs, L, dL);
    upload_dense(It64, It32, L);
}

// lanes per row of a transfer: FP32 (the multigrid's own precision) reads long
// rows with lane groups; FP64 keeps one thread per row, whose sums run over
// the row in order (the exact-parity path: its iteration counts match the
// oracle's, and a reordered sum can flip a line-search decision on a knife
// edge)
template <typename T> static int lanes(const DevCsr &M)
{
    return std::is_same<T, float>::value ? kron_lanes(M.nnz, M.nrows) : 1;
}

template <typename T> static const T *pick(const DevBuf &b64, const DevBuf &b32)
{
    return std::is_same<T, double>::value ? (const T *)b64.p : (const T *)b32.p;
}

template <typename T>
void Transfer::prolongate(const Level &f, const Level &c, const T *xc, T *yf, T beta, hipStream_t s) const
{
    KronCsrArgs<T> a{};
    a.rowptr = vel.rowptr.as<int>();
    a.col = vel.col.as<int>();
    a.val = pick<T>(vel.val64, vel.val32);
    a.nrows = vel.nrows;
    a.lpr = lanes<T>(vel);
    a.nt_out = f.nt;
    a.nt_in = c.nt;
    a.ncomp = f.dim;
    a.Tm = pick<T>(Pt64, Pt32);
    a.in_t_stride = c.Nv1;
    a.in_c_stride = c.Nn;
    a.out_t_stride = f.Nv1;
    a.out_c_stride = f.Nn;
    a.x = xc;
    a.y = yf;
    a.beta = beta;
    STMG_HIP(kron_csr_apply<T>(a, s));
    a.rowptr = pres.rowptr.as<int>();
    a.col = pres.col.as<int>();
    a.val = pick<T>(pres.val64, pres.val32);
    a.nrows = pres.nrows;
    a.lpr = lanes<T>(pres);
    a.ncomp = 1;
    a.in_t_stride = c.Np1;
    a.in_c_stride = 0;
    a.out_t_stride = f.Np1;
    a.out_c_stride = 0;
    a.x = xc + c.nt * c.Nv1;
    a.y = yf + f.nt * f.Nv1;
    STMG_HIP(kron_csr_apply<T>(a, s));
}

template <typename T>
void Transfer::restrict_(const Level &f, const Level &c, const T *xf, T *yc, hipStream_t s) const
{
    KronCsrArgs<T> a{};
    a.rowptr = velT.rowptr.as<int>();
    a.col = velT.col.as<int>();
    a.val = pick<T>(velT.val64, velT.val32);
    a.nrows = velT.nrows;
    a.lpr = lanes<T>(velT);
    a.nt_out = c.nt;
    a.nt_in = f.nt;
    a.ncomp = f.dim;
    a.Tm = pick<T>(PtT64, PtT32);
    a.in_t_stride = f.Nv1;
    a.in_c_stride = f.Nn;
    a.out_t_stride = c.Nv1;
    a.out_c_stride = c.Nn;
    a.x = xf;
    a.y = yc;
    a.beta = 0;
    STMG_HIP(kron_csr_apply<T>(a, s));
    a.rowptr = presT.rowptr.as<int>();
    a.col = presT.col.as<int>();
    a.val = pick<T>(presT.val64, presT.val32);
    a.nrows = presT.nrows;
    a.lpr = lanes<T>(presT);
    a.ncomp = 1;
    a.in_t_stride = f.Np1;
    a.in_c_stride = 0;
    a.out_t_stride = c.Np1;
    a.out_c_stride = 0;
    a.x = xf + f.nt * f.Nv1;
    a.y = yc + c.nt * c.Nv1;
    STMG_HIP(kron_csr_apply<T>(a, s));
}

template <typename T>
void Transfer::interpolate_state(const Level &f, const Level &c, const T *vf, T *vc, hipStream_t s) const
{
    KronCsrArgs<T> a{};
    a.rowptr = state.rowptr.as<int>();
    a.col = state.col.as<int>();
    a.val = pick<T>(state.val64, state.val32);
    a.nrows = state.nrows;
    a.lpr = lanes<T>(state);
    a.nt_out = c.nt;
    a.nt_in = f.nt;
    a.ncomp = f.dim;
    a.Tm = pick<T>(It64, It32);
    a.in_t_stride = f.Nv1;
    a.in_c_stride = f.Nn;
    a.out_t_stride = c.Nv1;
    a.out_c_stride = c.Nn;
    a.x = vf;
    a.y = vc;
    a.beta = 0;
    STMG_HIP(kron_csr_apply<T>(a, s));
}

template void Transfer::prolongate<double>(const Level &, const Level &, const double *, double *, double,
                                           hipStream_t) const;
template void Transfer::prolongate<float>(const Level &, const Level &, const float *, float *, float,
                                          hipStream_t) const;
template void Transfer::restrict_<double>(const Level &, const Level &, const double *, double *, hipStream_t) const;
template void Transfer::restrict_<float>(const Level &, const Level &, const float *, float *, hipStream_t) const;
template void Transfer::interpolate_state<double>(const Level &, const Level &, const double *, double *,
                                                  hipStream_t) const;
template void Transfer::interpolate_state<float>(const Level &, const Level &, const float *, float *,
                                                 hipStream_t) const;

} // namespace stmg
