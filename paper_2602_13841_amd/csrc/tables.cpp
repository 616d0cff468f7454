// One-dimensional tables of the space-time discretization, computed on the
// host when a context or level is created.
//
// * Gauss-Legendre rules: Newton iteration on P_n from Chebyshev guesses.
// * Gauss-Lobatto points (velocity nodes of Q_{r+1}): end points plus the
//   roots of P'_N, by Newton iteration with the Legendre ODE for P''_N.
// * Right Gauss-Radau rule with k+1 points (last node +1, exact for degree
//   2k; Sec. "Preliminaries", eq. GF): roots of P_{k+1} - P_k by Newton,
//   weights (1 + x)/((k+1)^2 P_k(x)^2) and 2/(k+1)^2 at x = +1.
// * Lagrange bases by the barycentric formula.
// * Time matrices of eq. DefKMC on the reference slab (K is independent of
//   tau; M = diag(tau/2 omega)).
// * Mapped P_r^disc pressure basis: orthonormal shifted Legendre products of
//   total degree <= r on the reference cell, first index fastest.
#include "stmg_internal.h"

#include <cmath>
#include <stdexcept>

namespace stmg {

namespace {

// P_n(x) and P_n'(x) by the three-term recurrence
void legendre(int n, double x, double &p, double &dp)
{
    double p0 = 1.0, p1 = x;
    if (n == 0) { p = 1.0; dp = 0.0; return; }
    for (int m = 2; m <= n; ++m) {
        double p2 = ((2.0 * m - 1.0) * x * p1 - (m - 1.0) * p0) / m;
        p0 = p1;
        p1 = p2;
    }
    p = p1;
    // derivative from (1 - x^2) P_n' = n (P_{n-1} - x P_n), valid for |x| < 1
    if (std::fabs(x) < 1.0) dp = n * (p0 - x * p1) / (1.0 - x * x);
    else dp = (x > 0 ? 1.0 : (n % 2 ? 1.0 : -1.0)) * 0.5 * n * (n + 1.0);
}

} // namespace

void gauss_rule(int nq, std::vector<double> &x01, std::vector<double> &w01)
{
    x01.assign(nq, 0.0);
    w01.assign(nq, 0.0);
    for (int i = 0; i < nq; ++i) {
        double x = -std::cos(M_PI * (i + 0.75) / (nq + 0.5));
        double p, dp;
        for (int it = 0; it < 100; ++it) {
            legendre(nq, x, p, dp);
            double dx = p / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        legendre(nq, x, p, dp);
        x01[i] = 0.5 * (x + 1.0);
        w01[i] = 0.5 * 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

void lobatto_points(int npts, std::vector<double> &x01)
{
    int N = npts - 1;
    x01.assign(npts, 0.0);
    x01[0] = 0.0;
    x01[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double x = -std::cos(M_PI * i / N);
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(N, x, p, dp);
            // q = P_N', q' = P_N'' = (2x P_N' - N(N+1) P_N)/(1-x^2)
            double ddp = (2.0 * x * dp - N * (N + 1.0) * p) / (1.0 - x * x);
            double dx = dp / ddp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        x01[i] = 0.5 * (x + 1.0);
    }
}

void radau_right(int k, std::vector<double> &x, std::vector<double> &w)
{
    int n = k + 1;
    x.assign(n, 1.0);
    w.assign(n, 0.0);
    for (int j = 0; j < k; ++j) {
        double t = -std::cos(M_PI * (2.0 * j + 1.0) / (2.0 * k + 1.0));
        for (int it = 0; it < 200; ++it) {
            double pa, dpa, pb, dpb;
            legendre(n, t, pa, dpa);
            legendre(k, t, pb, dpb);
            double f = pa - pb, df = dpa - dpb;
            double dt = f / df;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        x[j] = t;
        double pk, dpk;
        legendre(k, t, pk, dpk);
        w[j] = (1.0 + t) / (double(n) * n * pk * pk);
    }
    x[k] = 1.0;
    w[k] = 2.0 / (double(n) * n);
}

// barycentric Lagrange values/derivatives: L[p*n + j] = ell_j(pts[p])
void lagrange_tables(const std::vector<double> &nodes, const std::vector<double> &pts,
                     std::vector<double> &L, std::vector<double> &dL)
{
    int n = (int)nodes.size(), np = (int)pts.size();
    std::vector<double> bw(n, 1.0);
    for (int j = 0; j < n; ++j)
        for (int m = 0; m < n; ++m)
            if (m != j) bw[j] /= (nodes[j] - nodes[m]);
    L.assign((size_t)np * n, 0.0);
    dL.assign((size_t)np * n, 0.0);
    for (int p = 0; p < np; ++p) {
        double x = pts[p];
        int hit = -1;
        for (int j = 0; j < n; ++j)
            if (x == nodes[j]) hit = j;
        if (hit >= 0) {
            // at a node: ell_j(x_i) = delta; ell_j'(x_i) = (bw_j/bw_i)/(x_i - x_j), diagonal by row sum zero
            for (int j = 0; j < n; ++j) L[p * n + j] = (j == hit) ? 1.0 : 0.0;
            double s = 0.0;
            for (int j = 0; j < n; ++j) {
                if (j == hit) continue;
                double v = (bw[j] / bw[hit]) / (nodes[hit] - nodes[j]);
                dL[p * n + j] = v;
                s += v;
            }
            dL[p * n + hit] = -s;
            continue;
        }
        // ell_j(x) = l(x) bw_j/(x - x_j), l(x) = prod (x - x_m)
        double l = 1.0;
        for (int m = 0; m < n; ++m) l *= (x - nodes[m]);
        double s1 = 0.0;
        for (int m = 0; m < n; ++m) s1 += 1.0 / (x - nodes[m]);
        for (int j = 0; j < n; ++j) {
            double ell = l * bw[j] / (x - nodes[j]);
            L[p * n + j] = ell;
            // ell_j' = ell_j * (sum_{m != j} 1/(x - x_m))
            dL[p * n + j] = ell * (s1 - 1.0 / (x - nodes[j]));
        }
    }
}

// sqrt(2i+1) P_i(2s-1), i = 0..r
void legendre01_table(int r, const std::vector<double> &pts, std::vector<double> &out)
{
    int np = (int)pts.size();
    out.assign((size_t)np * (r + 1), 0.0);
    for (int p = 0; p < np; ++p) {
        double x = 2.0 * pts[p] - 1.0;
        double p0 = 1.0, p1 = x;
        for (int i = 0; i <= r; ++i) {
            double val;
            if (i == 0) val = 1.0;
            else if (i == 1) val = x;
            else {
                double p2 = ((2.0 * i - 1.0) * x * p1 - (i - 1.0) * p0) / i;
                p0 = p1;
                p1 = p2;
                val = p2;
            }
            out[p * (r + 1) + i] = std::sqrt(2.0 * i + 1.0) * val;
        }
    }
}

std::vector<int> pressure_multi_indices(int r, int dim)
{
    std::vector<int> m;
    int z_hi = dim == 3 ? r : 0;
    for (int a2 = 0; a2 <= z_hi; ++a2)
        for (int a1 = 0; a1 <= r; ++a1)
            for (int a0 = 0; a0 <= r; ++a0)
                if (a0 + a1 + a2 <= r) {
                    m.push_back(a0);
                    m.push_back(a1);
                    m.push_back(a2);
                }
    return m;
}

TimeCoefs time_coefficients(int k, double tau)
{
    if (k < 0 || k > MAX_K) throw std::runtime_error("unsupported time degree k");
    TimeCoefs tc{};
    int n = k + 1;
    tc.nt = n;
    std::vector<double> xr, wr;
    radau_right(k, xr, wr);
    std::vector<double> s(n);
    for (int a = 0; a < n; ++a) s[a] = 0.5 * (xr[a] + 1.0);    // nodes on [0,1]
    // K_ab = int_0^1 phi_b' phi_a ds + phi_b(0) phi_a(0)   (scale invariant)
    std::vector<double> gx, gw;
    gauss_rule(n + 1, gx, gw);
    std::vector<double> L, dL, L0, dL0, Lm, dLm;
    lagrange_tables(s, gx, L, dL);
    lagrange_tables(s, std::vector<double>{0.0}, L0, dL0);
    lagrange_tables(s, std::vector<double>{0.5}, Lm, dLm);
    for (int a = 0; a < n; ++a) {
        for (int b = 0; b < n; ++b) {
            double v = 0.0;
            for (int g = 0; g < (int)gx.size(); ++g) v += gw[g] * dL[g * n + b] * L[g * n + a];
            tc.K[a * n + b] = v + L0[b] * L0[a];
        }
        tc.w[a] = 0.5 * tau * wr[a];
        tc.phi0[a] = L0[a];
        tc.phimid[a] = Lm[a];
        tc.s[a] = s[a];
    }
    return tc;
}

// Interpolation matrix of the DG(kc) time basis into DG(kf): P[a*nc + b] =
// phi^c_b(t^f_a) (canonical embedding of P_kc into P_kf).
std::vector<double> time_embedding(int kf, int kc)
{
    TimeCoefs f = time_coefficients(kf, 1.0), c = time_coefficients(kc, 1.0);
    std::vector<double> cs(c.s, c.s + c.nt), fs(f.s, f.s + f.nt), L, dL;
    lagrange_tables(cs, fs, L, dL);
    return L;
}

int default_nq(int r) { return (3 * r + 5) / 2; }

} // namespace stmg

namespace stmg {

std::vector<double> build_table_block(int r, int nq, const TableLayout &lay)
{
    int n1 = r + 2, rp1 = r + 1;
    std::vector<double> out(lay.total, 0.0);
    std::vector<double> gll, gx, gw, L, dL, Lq, dLq, Le, dLe, Pq, Pe;
    lobatto_points(n1, gll);
    gauss_rule(nq, gx, gw);
    lagrange_tables(gll, gx, L, dL);            // [q][i]
    lagrange_tables(gx, gx, Lq, dLq);           // collocation derivative [q][m]
    std::vector<double> ends{0.0, 1.0};
    lagrange_tables(gll, ends, Le, dLe);        // [s][i]
    legendre01_table(r, gx, Pq);                // [q][alpha]
    legendre01_table(r, ends, Pe);              // [s][alpha]
    for (int q = 0; q < nq; ++q)
        for (int i = 0; i < n1; ++i) {
            out[lay.S + q * n1 + i] = L[q * n1 + i];
            out[lay.St + i * nq + q] = L[q * n1 + i];
            out[lay.D + q * n1 + i] = dL[q * n1 + i];
            out[lay.Dt + i * nq + q] = dL[q * n1 + i];
        }
    for (int q = 0; q < nq; ++q)
        for (int m = 0; m < nq; ++m) {
            out[lay.Dq + q * nq + m] = dLq[q * nq + m];
            out[lay.Dqt + m * nq + q] = dLq[q * nq + m];
        }
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < n1; ++i) {
            out[lay.Se + s * n1 + i] = Le[s * n1 + i];
            out[lay.De + s * n1 + i] = dLe[s * n1 + i];
        }
    for (int q = 0; q < nq; ++q)
        for (int a = 0; a < rp1; ++a) {
            out[lay.L + q * rp1 + a] = Pq[q * rp1 + a];
            out[lay.Lt + a * nq + q] = Pq[q * rp1 + a];
        }
    for (int s = 0; s < 2; ++s)
        for (int a = 0; a < rp1; ++a) out[lay.Le + s * rp1 + a] = Pe[s * rp1 + a];
    for (int q = 0; q < nq; ++q) out[lay.qw + q] = gw[q];
    for (int q = 0; q < nq; ++q) out[lay.qx + q] = gx[q];
    return out;
}

} // namespace stmg

// ---------------------------------------------------------------------------
// Diagonalization of the time coupling of the midpoint-surrogate patch
// ---------------------------------------------------------------------------
#include <complex>

namespace stmg {

namespace {

using cplx = std::complex<double>;

// Gaussian elimination with complete pivoting on an n x n complex matrix of
// rank n-1: returns a null vector normalized to largest component 1.
std::vector<cplx> null_vector(std::vector<cplx> B, int n)
{
    std::vector<int> colp(n);
    for (int j = 0; j < n; ++j) colp[j] = j;
    for (int c = 0; c < n - 1; ++c) {
        int pr = c, pc = c;
        double best = -1.0;
        for (int i = c; i < n; ++i)
            for (int j = c; j < n; ++j)
                if (std::abs(B[i * n + j]) > best) {
                    best = std::abs(B[i * n + j]);
                    pr = i;
                    pc = j;
                }
        for (int j = 0; j < n; ++j) std::swap(B[c * n + j], B[pr * n + j]);
        for (int i = 0; i < n; ++i) std::swap(B[i * n + c], B[i * n + pc]);
        std::swap(colp[c], colp[pc]);
        for (int i = c + 1; i < n; ++i) {
            cplx l = B[i * n + c] / B[c * n + c];
            for (int j = c; j < n; ++j) B[i * n + j] -= l * B[c * n + j];
        }
    }
    // the last permuted unknown is free (= 1); back substitution for the rest
    std::vector<cplx> y(n);
    y[n - 1] = 1.0;
    for (int i = n - 2; i >= 0; --i) {
        cplx s = 0.0;
        for (int j = i + 1; j < n; ++j) s += B[i * n + j] * y[j];
        y[i] = -s / B[i * n + i];
    }
    std::vector<cplx> v(n);
    for (int j = 0; j < n; ++j) v[colp[j]] = y[j];
    cplx big = 0.0;
    for (int j = 0; j < n; ++j)
        if (std::abs(v[j]) > std::abs(big)) big = v[j];
    for (int j = 0; j < n; ++j) v[j] /= big;
    return v;
}

// inverse of an n x n complex matrix (partial pivoting)
std::vector<cplx> inverse(std::vector<cplx> A, int n)
{
    std::vector<cplx> X(n * n, 0.0);
    for (int i = 0; i < n; ++i) X[i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int i = c + 1; i < n; ++i)
            if (std::abs(A[i * n + c]) > std::abs(A[p * n + c])) p = i;
        for (int j = 0; j < n; ++j) {
            std::swap(A[c * n + j], A[p * n + j]);
            std::swap(X[c * n + j], X[p * n + j]);
        }
        const cplx d = A[c * n + c];
        if (d == cplx(0.0)) throw std::runtime_error("singular eigenvector matrix of the time coupling");
        for (int j = 0; j < n; ++j) {
            A[c * n + j] /= d;
            X[c * n + j] /= d;
        }
        for (int i = 0; i < n; ++i) {
            if (i == c) continue;
            const cplx l = A[i * n + c];
            for (int j = 0; j < n; ++j) {
                A[i * n + j] -= l * A[c * n + j];
                X[i * n + j] -= l * X[c * n + j];
            }
        }
    }
    return X;
}

} // namespace

// The surrogate patch of eq. DefTildeHn has the Kronecker form
//   K (x) Mhat + W (x) Ahat = (W (x) I) (E (x) Mhat + I (x) Ahat),  E = W^{-1} K,
// with Mhat the velocity mass and Ahat the shared spatial core.  With
// E = S diag(lambda) S^{-1} the patch solve splits into one spatial solve per
// eigenvalue, (lambda Mhat + Ahat) z = (S^{-1} W^{-1} r)_lambda; a conjugate
// pair needs one complex solve.  Eigenvalues are the roots of the
// characteristic polynomial (Faddeev-LeVerrier coefficients, Durand-Kerner
// iteration, Newton polish), eigenvectors the null vectors of E - lambda I.
TimeDiag time_diagonalization(const TimeCoefs &tc)
{
    const int n = tc.nt;
    TimeDiag td{};
    std::vector<double> E(n * n);
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) E[a * n + b] = tc.K[a * n + b] / tc.w[a];
    // characteristic polynomial p(x) = x^n + c[n-1] x^{n-1} + ... + c[0]
    std::vector<double> c(n + 1, 0.0), Mk(n * n, 0.0), AM(n * n);
    c[n] = 1.0;
    for (int k = 1; k <= n; ++k) {
        // M_k = E M_{k-1} + c_{n-k+1} I, c_{n-k} = -tr(E M_k) / k
        std::vector<double> Mn(n * n, 0.0);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int l = 0; l < n; ++l) s += E[i * n + l] * Mk[l * n + j];
                Mn[i * n + j] = s + (i == j ? c[n - k + 1] : 0.0);
            }
        Mk = Mn;
        double tr = 0.0;
        for (int i = 0; i < n; ++i)
            for (int l = 0; l < n; ++l) tr += E[i * n + l] * Mk[l * n + i];
        c[n - k] = -tr / k;
    }
    auto poly = [&](cplx x) {
        cplx v = 1.0;
        for (int k = n - 1; k >= 0; --k) v = v * x + c[k];
        return v;
    };
    auto dpoly = [&](cplx x) {
        cplx v = double(n);
        for (int k = n - 1; k >= 1; --k) v = v * x + double(k) * c[k];
        return v;
    };
    double scale = 0.0;
    for (int i = 0; i < n * n; ++i) scale = std::max(scale, std::abs(E[i]));
    std::vector<cplx> z(n);
    for (int i = 0; i < n; ++i) z[i] = scale * std::pow(cplx(0.4, 0.9), i);
    for (int it = 0; it < 500; ++it) {
        double move = 0.0;
        for (int i = 0; i < n; ++i) {
            cplx den = 1.0;
            for (int j = 0; j < n; ++j)
                if (j != i) den *= (z[i] - z[j]);
            cplx dz = poly(z[i]) / den;
            z[i] -= dz;
            move = std::max(move, std::abs(dz));
        }
        if (move <= 1e-15 * scale) break;
    }
    for (int i = 0; i < n; ++i)
        for (int it = 0; it < 3; ++it) {
            cplx d = dpoly(z[i]);
            if (d != cplx(0.0)) z[i] -= poly(z[i]) / d;
        }
    // order: real eigenvalues, then one member (Im > 0) of each conjugate pair
    std::vector<cplx> lam;
    for (int i = 0; i < n; ++i)
        if (std::fabs(z[i].imag()) <= 1e-10 * std::abs(z[i])) lam.push_back(cplx(z[i].real(), 0.0));
    const int nreal = (int)lam.size();
    for (int i = 0; i < n; ++i)
        if (z[i].imag() > 1e-10 * std::abs(z[i])) lam.push_back(z[i]);
    if (nreal + 2 * ((int)lam.size() - nreal) != n) throw std::runtime_error("time coupling eigenvalues not paired");
    // eigenvector matrix S: columns per system (pairs: v, conj v)
    std::vector<cplx> S(n * n);
    std::vector<int> col_of(lam.size());
    int col = 0;
    for (size_t s = 0; s < lam.size(); ++s) {
        std::vector<cplx> B(n * n);
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) B[a * n + b] = E[a * n + b] - (a == b ? lam[s] : 0.0);
        std::vector<cplx> v = null_vector(B, n);
        if ((int)s < nreal)
            for (int a = 0; a < n; ++a) v[a] = cplx(v[a].real(), 0.0);
        col_of[s] = col;
        for (int a = 0; a < n; ++a) S[a * n + col] = v[a];
        ++col;
        if ((int)s >= nreal) {
            for (int a = 0; a < n; ++a) S[a * n + col] = std::conj(v[a]);
            ++col;
        }
    }
    std::vector<cplx> Si = inverse(S, n);
    // check E S = S Lambda
    double err = 0.0, ref = 0.0;
    for (int a = 0; a < n; ++a)
        for (int j = 0; j < n; ++j) {
            cplx es = 0.0;
            for (int b = 0; b < n; ++b) es += E[a * n + b] * S[b * n + j];
            cplx lj = 0.0;
            for (size_t s = 0; s < lam.size(); ++s) {
                if (col_of[s] == j) lj = lam[s];
                if ((int)s >= nreal && col_of[s] + 1 == j) lj = std::conj(lam[s]);
            }
            err = std::max(err, std::abs(es - S[a * n + j] * lj));
            ref = std::max(ref, std::abs(es));
        }
    if (!(err <= 1e-10 * std::max(ref, 1e-300))) throw std::runtime_error("time coupling diagonalization inaccurate");
    td.nsys = (int)lam.size();
    for (int s = 0; s < td.nsys; ++s) {
        td.cplx[s] = s >= nreal ? 1 : 0;
        td.lre[s] = lam[s].real();
        td.lim[s] = lam[s].imag();
        const int j = col_of[s];
        const double f = td.cplx[s] ? 2.0 : 1.0;
        for (int a = 0; a < n; ++a) {
            cplx t = Si[j * n + a] / tc.w[a];
            td.Tre[s * MAX_NT + a] = t.real();
            td.Tim[s * MAX_NT + a] = t.imag();
            td.Fre[a * MAX_NT + s] = f * S[a * n + j].real();
            td.Fim[a * MAX_NT + s] = f * S[a * n + j].imag();
        }
    }
    return td;
}

} // namespace stmg
